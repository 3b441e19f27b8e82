// libpstd C ABI, DCT-basis neural-operator surrogate: parameters, forward, backward, Adam.
//
// The network (features -> lift -> layers of GELU(W v + b + IDCT(R . DCT(v))) -> two-layer projection)
// runs as a sequence of nop_gemm launches whose strides express every contraction in place; the
// orthonormal DCT-II matrices of the retained modes are built here in FP64 and kept in FP32.  All
// buffers are sized for the configured maximum batch at creation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

struct pstd_nop_s {
  pstd_nop_config cfg{};
  hipStream_t stream = nullptr;
  int64_t P = 0, nparam = 0;
  int64_t oP = 0, opb = 0, oR[16] = {}, oW[16] = {}, ob[16] = {}, oQ1 = 0, oq1b = 0, oQ2 = 0, oq2b = 0;
  float *theta = nullptr, *grad = nullptr, *m1 = nullptr, *m2 = nullptr;
  int64_t adam_t = 0;
  float *Ch = nullptr, *Cw = nullptr;
  void *dct2_img = nullptr, *idct_img = nullptr;   // bf16 LDS images of the tables
  float* F = nullptr;
  std::vector<float*> V, PRE, AT;
  float *qpre = nullptr, *q = nullptr, *out = nullptr;
  float *Y1 = nullptr, *Ahat = nullptr, *Zt = nullptr, *At2 = nullptr, *T = nullptr;
  float *dv = nullptr, *dvn = nullptr, *dpre = nullptr, *dq = nullptr, *dout = nullptr, *part = nullptr;
  double* terms = nullptr;
  std::vector<void*> owned;
  int last_batch = 0;
  bool have_fwd = false;
};

namespace pstd {
namespace {

int nop_alloc(pstd_nop_s* N, void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) return fail(PSTD_E_OOM, "hipMalloc of %zu bytes failed", bytes);
  N->owned.push_back(*p);
  return PSTD_OK;
}

void nop_free(pstd_nop_s* N) {
  if (!N) return;
  for (void* p : N->owned) (void)hipFree(p);
  delete N;
}

std::vector<double> dct_rows(int n, int m) {
  std::vector<double> c(static_cast<size_t>(m) * n);
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < n; ++j)
      c[static_cast<size_t>(k) * n + j] =
          (k == 0 ? std::sqrt(1.0 / n) : std::sqrt(2.0 / n)) * std::cos(M_PI * k * (2.0 * j + 1.0) / (2.0 * n));
  return c;
}

NopGemm gemm(const pstd_nop_s* Nn, const float* A, int64_t sAm, int64_t sAk, const float* B, int64_t sBk,
             int64_t sBn, float* C, int64_t sCm, int64_t sCn, int M, int N, int K) {
  NopGemm g{};
  g.A = A;
  g.B = B;
  g.C = C;
  g.M = M;
  g.N = N;
  g.K = K;
  g.sAm = sAm;
  g.sAk = sAk;
  g.sBk = sBk;
  g.sBn = sBn;
  g.sCm = sCm;
  g.sCn = sCn;
  g.nb1 = 1;
  g.nb2 = 1;
  g.alpha = 1.f;
  g.beta = 0.f;
  g.split = Nn->cfg.split;
  return g;
}

// Split of the P positions into chunks for weight-gradient products (batch x chunk partial sums).
int chunks_of(int64_t P) {
  for (int c : {16, 8, 4, 2})
    if (P % c == 0 && P / c >= 32) return c;
  return 1;
}

#define NOP_RUN(expr)                                                                                 \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess) return fail(PSTD_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

// Spectral term of one layer up to its last stage: T = (inverse DCT along H of) R . DCT(vin), laid out
// [b][h][c][kw]; keeps the blocked DCT in `at`.
int spectral_fwd(pstd_nop_s* N, const void* vin, const float* R, float* at, int B, bool half) {
  const pstd_nop_config& c = N->cfg;
  const int H = c.H, W = c.W, C = c.channels, Mm = c.modes;
  const int64_t P = N->P;
  hipStream_t s = N->stream;
  NopGemm g;
  if (nop_dct2_supported(H, W, Mm)) {
    // both DCT stages per plane in registers: Ahat[b][c] = Ch vin[b][c] Cw^T
    NOP_RUN(launch_nop_dct2(vin, N->Ahat, N->dct2_img, B * C, H, W, Mm, c.split != 0, half, s));
  } else {
    // DCT along H: Y1[bc] (Mm x W) = Ch (Mm x H) vin[bc] (H x W)
    g = gemm(N, N->Ch, H, 1, static_cast<const float*>(vin), W, 1, N->Y1, W, 1, Mm, W, H);
    g.nb1 = B * C;
    g.bB1 = P;
    g.bC1 = static_cast<int64_t>(Mm) * W;
    NOP_RUN(launch_nop_gemm(g, s));
    // DCT along W: Ahat[(bc,kh)][kw] = sum_w Y1[(bc,kh)][w] Cw[kw][w]
    g = gemm(N, N->Y1, W, 1, N->Cw, 1, W, N->Ahat, Mm, 1, B * C * Mm, Mm, W);
    NOP_RUN(launch_nop_gemm(g, s));
  }
  NOP_RUN(launch_nop_mode_transpose(N->Ahat, at, B, C, Mm, true, s));
  // mixing per 2 x 2 mode block: Zt[blk] (4B x C) = at[blk] (4B x C) R[blk]^T
  g = gemm(N, at, C, 1, R, 1, C, N->Zt, C, 1, 4 * B, C, C);
  g.nb1 = (Mm / 2) * (Mm / 2);
  g.bA1 = 4LL * B * C;
  g.bB1 = static_cast<int64_t>(C) * C;
  g.bC1 = 4LL * B * C;
  NOP_RUN(launch_nop_gemm(g, s));
  NOP_RUN(launch_nop_mode_transpose(N->Zt, N->Ahat, B, C, Mm, false, s));
  // inverse along H: T[b][h][c][kw] = sum_kh Ch[kh][h] Z[b][c][kh][kw]; the inverse along W is the
  // second K segment of the channel-mixing kernel that consumes T
  if (Mm <= 64 && H <= 512) {
    NOP_RUN(launch_nop_idct_h(N->Ahat, N->T, N->idct_img, B, C, H, Mm, c.split != 0, half, s));
  } else {
    g = gemm(N, N->Ch, 1, H, N->Ahat, Mm, 1, N->T, static_cast<int64_t>(C) * Mm, 1, H, Mm, Mm);
    g.nb1 = B;
    g.bB1 = static_cast<int64_t>(C) * Mm * Mm;
    g.bC1 = static_cast<int64_t>(H) * C * Mm;
    g.nb2 = C;
    g.bB2 = static_cast<int64_t>(Mm) * Mm;
    g.bC2 = Mm;
    NOP_RUN(launch_nop_gemm(g, s));
  }
  return PSTD_OK;
}

// Weight gradient G (M x Nc) = sum_b sum_p X[b][m][p] Y[b][n][p] through batch x chunk partials.
int weight_grad(pstd_nop_s* N, const float* X, int M, const float* Y, int Nc, float* G, int B) {
  const int64_t P = N->P;
  const int nch = chunks_of(P);
  const int64_t KC = P / nch;
  NopGemm g = gemm(N, X, P, 1, Y, 1, P, N->part, Nc, 1, M, Nc, static_cast<int>(KC));
  g.nb1 = B;
  g.nb2 = nch;
  g.bA1 = static_cast<int64_t>(M) * P;
  g.bA2 = KC;
  g.bB1 = static_cast<int64_t>(Nc) * P;
  g.bB2 = KC;
  g.bC1 = static_cast<int64_t>(nch) * M * Nc;
  g.bC2 = static_cast<int64_t>(M) * Nc;
  NOP_RUN(launch_nop_gemm(g, N->stream));
  NOP_RUN(launch_nop_partial_sum(N->part, G, B * nch, M * Nc, N->stream));
  return PSTD_OK;
}

}  // namespace
}  // namespace pstd

using namespace pstd;

extern "C" {

int pstd_nop_create(const pstd_nop_config* cfg, void* hip_stream, pstd_nop* out) {
  if (!out) return fail(PSTD_E_INVALID_ARG, "out is null");
  *out = nullptr;
  if (!cfg) return fail(PSTD_E_INVALID_ARG, "cfg is null");
  const pstd_nop_config c = *cfg;
  if (c.H < 2 || c.W < 2 || c.channels < 1 || c.channels > 32 || c.modes < 2 || c.modes % 2 || c.modes > c.H ||
      c.modes > c.W || c.modes > 256 ||
      c.layers < 1 || c.layers > 16 || c.hidden < 1 || c.hidden > 256 || c.max_batch < 1 || (c.split != 0 && c.split != 1))
    return fail(PSTD_E_INVALID_ARG, "bad surrogate configuration");
  const int64_t P = static_cast<int64_t>(c.H) * c.W;
  const int64_t B = c.max_batch;
  if (B * c.channels * P >= (int64_t(1) << 31) || B * c.hidden * P >= (int64_t(1) << 31))
    return fail(PSTD_E_UNSUPPORTED, "activation tensors above 2^31 elements");
  if (B * c.channels > 65535 || static_cast<int64_t>(c.modes / 2) * (c.modes / 2) > 65535 || B * 16 > 65535)
    return fail(PSTD_E_UNSUPPORTED, "batch too large for the launch grid");
  pstd_nop_s* N = new pstd_nop_s();
  N->cfg = c;
  N->stream = static_cast<hipStream_t>(hip_stream);
  N->P = P;
  const int C = c.channels, Mm = c.modes, Hp = c.hidden;
  int64_t o = 0;
  N->oP = o; o += 4LL * C;
  N->opb = o; o += C;
  for (int l = 0; l < c.layers; ++l) {
    N->oR[l] = o; o += static_cast<int64_t>(Mm / 2) * (Mm / 2) * C * C;
    N->oW[l] = o; o += static_cast<int64_t>(C) * C;
    N->ob[l] = o; o += C;
  }
  N->oQ1 = o; o += static_cast<int64_t>(Hp) * C;
  N->oq1b = o; o += Hp;
  N->oQ2 = o; o += Hp;
  N->oq2b = o; o += 1;
  N->nparam = o;
  const int64_t act = B * C * P;
  const int64_t spec = B * C * static_cast<int64_t>(Mm) * Mm;
  const int64_t ysz = B * C * static_cast<int64_t>(Mm) * std::max(c.H, c.W);
  const int nch = chunks_of(P);
  const int64_t partsz = B * nch * std::max<int64_t>(static_cast<int64_t>(Hp) * C, static_cast<int64_t>(C) * C);
  int st = PSTD_OK;
  auto A = [&](float** p, int64_t n) {
    if (st == PSTD_OK) st = nop_alloc(N, reinterpret_cast<void**>(p), static_cast<size_t>(n) * sizeof(float));
  };
  A(&N->theta, o);
  A(&N->grad, o);
  A(&N->m1, o);
  A(&N->m2, o);
  A(&N->Ch, static_cast<int64_t>(Mm) * c.H);
  A(&N->Cw, static_cast<int64_t>(Mm) * c.W);
  A(&N->F, B * 4 * P);
  N->V.assign(c.layers + 1, nullptr);
  N->PRE.assign(c.layers, nullptr);
  N->AT.assign(c.layers, nullptr);
  for (int l = 0; l <= c.layers; ++l) A(&N->V[l], act);
  for (int l = 0; l < c.layers; ++l) {
    A(&N->PRE[l], act);
    A(&N->AT[l], spec);
  }
  A(&N->qpre, B * Hp * P);
  A(&N->q, B * Hp * P);
  A(&N->out, B * P);
  A(&N->Y1, ysz);
  A(&N->Ahat, spec);
  A(&N->Zt, spec);
  A(&N->At2, spec);
  A(&N->T, B * c.H * C * Mm);
  A(&N->dv, act);
  A(&N->dvn, act);
  A(&N->dpre, act);
  A(&N->dq, B * Hp * P);
  A(&N->dout, B * P);
  A(&N->part, partsz);
  if (st == PSTD_OK && nop_alloc(N, reinterpret_cast<void**>(&N->terms), 2 * B * sizeof(double)) != PSTD_OK)
    st = PSTD_E_OOM;
  if (st != PSTD_OK) {
    nop_free(N);
    return st;
  }
  // DCT matrices, FP64 -> FP32
  for (int ax = 0; ax < 2; ++ax) {
    const int n = ax == 0 ? c.H : c.W;
    const std::vector<double> d = dct_rows(n, Mm);
    std::vector<float> f(d.begin(), d.end());
    if (hipMemcpy(ax == 0 ? N->Ch : N->Cw, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
      nop_free(N);
      return fail(PSTD_E_HIP, "copy of the DCT matrices failed");
    }
  }
  {
    size_t db = 0, ib = 0;
    nop_table_bytes(c.H, c.W, Mm, c.split != 0, &db, &ib);
    if (nop_alloc(N, &N->dct2_img, db) != PSTD_OK || nop_alloc(N, &N->idct_img, ib) != PSTD_OK) {
      nop_free(N);
      return PSTD_E_OOM;
    }
    if (launch_nop_tables(N->Ch, N->Cw, N->dct2_img, N->idct_img, c.H, c.W, Mm, c.split != 0, N->stream) != hipSuccess ||
        hipStreamSynchronize(N->stream) != hipSuccess) {
      nop_free(N);
      return fail(PSTD_E_HIP, "building the DCT table images failed");
    }
  }
  if (hipMemset(N->theta, 0, o * sizeof(float)) != hipSuccess || hipMemset(N->m1, 0, o * sizeof(float)) != hipSuccess ||
      hipMemset(N->m2, 0, o * sizeof(float)) != hipSuccess || hipMemset(N->grad, 0, o * sizeof(float)) != hipSuccess) {
    nop_free(N);
    return fail(PSTD_E_HIP, "hipMemset failed");
  }
  *out = N;
  return PSTD_OK;
}

int64_t pstd_nop_param_count(pstd_nop N) { return N ? N->nparam : -1; }

int pstd_nop_set_params(pstd_nop N, const float* host, int64_t n) {
  if (!N || !host || n != N->nparam) return fail(PSTD_E_INVALID_ARG, "null handle/pointer or wrong count");
  PSTD_HIP(hipMemcpy(N->theta, host, n * sizeof(float), hipMemcpyHostToDevice));
  PSTD_HIP(hipMemset(N->m1, 0, n * sizeof(float)));
  PSTD_HIP(hipMemset(N->m2, 0, n * sizeof(float)));
  N->adam_t = 0;
  return PSTD_OK;
}

int pstd_nop_get_params(pstd_nop N, float* host, int64_t n) {
  if (!N || !host || n != N->nparam) return fail(PSTD_E_INVALID_ARG, "null handle/pointer or wrong count");
  PSTD_HIP(hipStreamSynchronize(N->stream));
  PSTD_HIP(hipMemcpy(host, N->theta, n * sizeof(float), hipMemcpyDeviceToHost));
  return PSTD_OK;
}

int pstd_nop_get_grads(pstd_nop N, float* host, int64_t n) {
  if (!N || !host || n != N->nparam) return fail(PSTD_E_INVALID_ARG, "null handle/pointer or wrong count");
  PSTD_HIP(hipStreamSynchronize(N->stream));
  PSTD_HIP(hipMemcpy(host, N->grad, n * sizeof(float), hipMemcpyDeviceToHost));
  return PSTD_OK;
}

}  // extern "C"

namespace pstd {
namespace {

// Forward pass; with keep every activation the backward pass needs is stored, otherwise the layers
// ping-pong between two buffers and nothing else is written.
int forward_impl(pstd_nop N, const float* p0, const float* c0, float* out, int32_t batch, bool keep) {
  if (!N || !p0 || !c0 || !out) return fail(PSTD_E_INVALID_ARG, "null pointer");
  if (batch < 1 || batch > N->cfg.max_batch) return fail(PSTD_E_INVALID_ARG, "batch must be 1..%d", N->cfg.max_batch);
  const pstd_nop_config& c = N->cfg;
  const int B = batch, C = c.channels, Hp = c.hidden;
  const int64_t P = N->P;
  hipStream_t s = N->stream;
  const float* th = N->theta;
  NOP_RUN(launch_nop_features(p0, c0, N->F, B, c.H, c.W, s));
  // lift: V0[b] (C x P) = Pw (C x 4) F[b] (4 x P) + pb
  // Inference without split keeps the activations (each layer's field and the first inverse stage T) in
  // bf16: every consumer rounds them to bf16 before its product, so the output is the same as with FP32
  // storage while the traffic of the dominant tensors halves.  Training and split keep FP32.
  const bool half = !keep && c.split == 0 && nop_dct2_supported(c.H, c.W, c.modes) && c.modes <= 64 && c.H <= 512;
  NOP_RUN(launch_nop_mix(th + N->oP, false, N->F, N->V[0], th + N->opb, nullptr, nullptr, nullptr, nullptr, 0, C, 4,
                         c.H, c.W, B, false, c.split != 0, half ? 1 : 0, s));
  float* vin = N->V[0];
  for (int l = 0; l < c.layers; ++l) {
    float* vout = keep ? N->V[l + 1] : N->V[(l + 1) & 1];
    const int st = spectral_fwd(N, vin, th + N->oR[l], keep ? N->AT[l] : N->At2, B, half);
    if (st != PSTD_OK) return st;
    // vout = GELU(W vin + b + S), pre-activation kept for the backward pass
    NOP_RUN(launch_nop_mix(th + N->oW[l], false, vin, vout, th + N->ob[l], nullptr, keep ? N->PRE[l] : nullptr, N->T,
                           N->Cw, c.modes, C, C, c.H, c.W, B, true, c.split != 0, half ? 2 : 0, s));
    vin = vout;
  }
  // projection: out = Q2 GELU(Q1 v + q1b) + q2b
  NOP_RUN(launch_nop_project(th + N->oQ1, th + N->oq1b, th + N->oQ2, th + N->oq2b, vin, N->out,
                             keep ? N->qpre : nullptr, keep ? N->q : nullptr, C, Hp, P, B, c.split != 0, half, s));
  if (out != N->out)
    PSTD_HIP(hipMemcpyAsync(out, N->out, static_cast<size_t>(B) * P * sizeof(float), hipMemcpyDeviceToDevice, s));
  N->last_batch = B;
  N->have_fwd = keep;
  return PSTD_OK;
}

}  // namespace
}  // namespace pstd

extern "C" {

int pstd_nop_forward(pstd_nop N, const float* p0, const float* c0, float* out, int32_t batch) {
  return forward_impl(N, p0, c0, out, batch, true);
}

int pstd_nop_infer(pstd_nop N, const float* p0, const float* c0, float* out, int32_t batch) {
  return forward_impl(N, p0, c0, out, batch, false);
}

int pstd_nop_backward(pstd_nop N, const float* target, double* loss) {
  if (!N || !target) return fail(PSTD_E_INVALID_ARG, "null pointer");
  if (!N->have_fwd) return fail(PSTD_E_INVALID_ARG, "backward needs a preceding forward");
  const pstd_nop_config& c = N->cfg;
  const int B = N->last_batch, C = c.channels, Hp = c.hidden, Mm = c.modes, H = c.H, W = c.W;
  const int64_t P = N->P;
  hipStream_t s = N->stream;
  const float* th = N->theta;
  float* gr = N->grad;
  NOP_RUN(launch_nop_loss(N->out, target, N->terms, N->dout, B, P, s));
  // output layer
  NOP_RUN(launch_nop_rowsum(N->dout, gr + N->oq2b, B, 1, P, s));
  int st = weight_grad(N, N->dout, 1, N->q, Hp, gr + N->oQ2, B);
  if (st != PSTD_OK) return st;
  // dq = (Q2 outer dout) * GELU'(qpre)
  NopGemm g = gemm(N, th + N->oQ2, 1, 1, N->dout, P, 1, N->dq, P, 1, Hp, static_cast<int>(P), 1);
  g.nb1 = B;
  g.bB1 = P;
  g.bC1 = Hp * P;
  g.dgelu = N->qpre;
  NOP_RUN(launch_nop_gemm(g, s));
  NOP_RUN(launch_nop_rowsum(N->dq, gr + N->oq1b, B, Hp, P, s));
  st = weight_grad(N, N->dq, Hp, N->V[c.layers], C, gr + N->oQ1, B);
  if (st != PSTD_OK) return st;
  // dv = Q1^T dq
  NOP_RUN(launch_nop_mix(th + N->oQ1, true, N->dq, N->dv, nullptr, nullptr, nullptr, nullptr, nullptr, 0, C, Hp, H, W,
                         B, false, c.split != 0, 0, s));
  for (int l = c.layers - 1; l >= 0; --l) {
    NOP_RUN(launch_nop_gelu_bwd(N->dv, N->PRE[l], N->dpre, static_cast<int64_t>(B) * C * P, s));
    NOP_RUN(launch_nop_rowsum(N->dpre, gr + N->ob[l], B, C, P, s));
    st = weight_grad(N, N->dpre, C, N->V[l], C, gr + N->oW[l], B);
    if (st != PSTD_OK) return st;
    // dvn = W^T dpre
    NOP_RUN(launch_nop_mix(th + N->oW[l], true, N->dpre, N->dvn, nullptr, nullptr, nullptr, nullptr, nullptr, 0, C, C,
                           H, W, B, false, c.split != 0, 0, s));
    // spectral path: dZ = DCT(dpre) (the inverse's adjoint), blocked
    g = gemm(N, N->Ch, H, 1, N->dpre, W, 1, N->Y1, W, 1, Mm, W, H);
    g.nb1 = B * C;
    g.bB1 = P;
    g.bC1 = static_cast<int64_t>(Mm) * W;
    NOP_RUN(launch_nop_gemm(g, s));
    g = gemm(N, N->Y1, W, 1, N->Cw, 1, W, N->Ahat, Mm, 1, B * C * Mm, Mm, W);
    NOP_RUN(launch_nop_gemm(g, s));
    NOP_RUN(launch_nop_mode_transpose(N->Ahat, N->Zt, B, C, Mm, true, s));
    // dR[blk] (C x C) = dZt[blk]^T (C x 4B) AT[l][blk] (4B x C)
    const int nblk = (Mm / 2) * (Mm / 2);
    g = gemm(N, N->Zt, 1, C, N->AT[l], C, 1, gr + N->oR[l], C, 1, C, C, 4 * B);
    g.nb1 = nblk;
    g.bA1 = 4LL * B * C;
    g.bB1 = 4LL * B * C;
    g.bC1 = static_cast<int64_t>(C) * C;
    NOP_RUN(launch_nop_gemm(g, s));
    // dA[blk] (4B x C) = dZt[blk] (4B x C) R[blk] (C x C)
    g = gemm(N, N->Zt, C, 1, th + N->oR[l], C, 1, N->At2, C, 1, 4 * B, C, C);
    g.nb1 = nblk;
    g.bA1 = 4LL * B * C;
    g.bB1 = static_cast<int64_t>(C) * C;
    g.bC1 = 4LL * B * C;
    NOP_RUN(launch_nop_gemm(g, s));
    NOP_RUN(launch_nop_mode_transpose(N->At2, N->Ahat, B, C, Mm, false, s));
    // dvn += IDCT(dA) (the DCT's adjoint)
    g = gemm(N, N->Ahat, Mm, 1, N->Cw, W, 1, N->Y1, W, 1, B * C * Mm, W, Mm);
    NOP_RUN(launch_nop_gemm(g, s));
    g = gemm(N, N->Ch, 1, H, N->Y1, W, 1, N->dvn, W, 1, H, W, Mm);
    g.nb1 = B * C;
    g.bB1 = static_cast<int64_t>(Mm) * W;
    g.bC1 = P;
    g.beta = 1.f;
    NOP_RUN(launch_nop_gemm(g, s));
    std::swap(N->dv, N->dvn);
  }
  // lift
  NOP_RUN(launch_nop_rowsum(N->dv, gr + N->opb, B, C, P, s));
  st = weight_grad(N, N->dv, C, N->F, 4, gr + N->oP, B);
  if (st != PSTD_OK) return st;
  if (loss) {
    std::vector<double> t(2 * B);
    PSTD_HIP(hipMemcpyAsync(t.data(), N->terms, 2 * B * sizeof(double), hipMemcpyDeviceToHost, s));
    PSTD_HIP(hipStreamSynchronize(s));
    double L = 0.0;
    for (int b = 0; b < B; ++b) L += t[2 * b] / t[2 * b + 1];
    *loss = L / B;
  }
  return PSTD_OK;
}

int pstd_nop_adam_step(pstd_nop N, double lr, double beta1, double beta2, double eps) {
  if (!N) return fail(PSTD_E_INVALID_ARG, "null handle");
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(PSTD_E_INVALID_ARG, "bad Adam hyper-parameters");
  N->adam_t += 1;
  const double c1 = 1.0 - std::pow(beta1, static_cast<double>(N->adam_t));
  const double c2 = 1.0 - std::pow(beta2, static_cast<double>(N->adam_t));
  NOP_RUN(launch_nop_adam(N->theta, N->grad, N->m1, N->m2, N->nparam, static_cast<float>(lr),
                          static_cast<float>(beta1), static_cast<float>(beta2), static_cast<float>(eps),
                          static_cast<float>(c1), static_cast<float>(c2), N->stream));
  return PSTD_OK;
}

int pstd_nop_relative_errors(pstd_nop N, const float* pred, const float* target, int32_t batch, double* err) {
  if (!N || !pred || !target || !err) return fail(PSTD_E_INVALID_ARG, "null pointer");
  if (batch < 1 || batch > N->cfg.max_batch) return fail(PSTD_E_INVALID_ARG, "bad batch");
  NOP_RUN(launch_nop_loss(pred, target, N->terms, nullptr, batch, N->P, N->stream));
  std::vector<double> t(2 * batch);
  PSTD_HIP(hipMemcpyAsync(t.data(), N->terms, 2 * batch * sizeof(double), hipMemcpyDeviceToHost, N->stream));
  PSTD_HIP(hipStreamSynchronize(N->stream));
  for (int b = 0; b < batch; ++b) err[b] = t[2 * b + 1] > 0 ? std::sqrt(t[2 * b] / t[2 * b + 1]) : 0.0;
  return PSTD_OK;
}

int pstd_nop_input_stats(pstd_nop N, const float* p0, const float* c0, int32_t batch, int32_t margin, double* stats) {
  if (!N || !p0 || !c0 || !stats) return fail(PSTD_E_INVALID_ARG, "null pointer");
  if (batch < 1 || batch > N->cfg.max_batch) return fail(PSTD_E_INVALID_ARG, "bad batch");
  if (margin < 0) return fail(PSTD_E_INVALID_ARG, "margin < 0");
  if (static_cast<int64_t>(4) * batch > 2LL * N->cfg.max_batch) {
    // terms holds 2 max_batch doubles; stats of larger batches go through a temporary buffer
    double* tmp = nullptr;
    if (hipMalloc(&tmp, 4 * sizeof(double) * batch) != hipSuccess) return fail(PSTD_E_OOM, "hipMalloc failed");
    hipError_t e = launch_nop_input_stats(p0, c0, tmp, batch, N->cfg.H, N->cfg.W, margin, N->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(stats, tmp, 4 * sizeof(double) * batch, hipMemcpyDeviceToHost, N->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(N->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(PSTD_E_HIP, "input statistics failed: %s", hipGetErrorString(e));
    return PSTD_OK;
  }
  NOP_RUN(launch_nop_input_stats(p0, c0, N->terms, batch, N->cfg.H, N->cfg.W, margin, N->stream));
  PSTD_HIP(hipMemcpyAsync(stats, N->terms, 4 * sizeof(double) * batch, hipMemcpyDeviceToHost, N->stream));
  PSTD_HIP(hipStreamSynchronize(N->stream));
  return PSTD_OK;
}

int pstd_nop_predict(pstd_nop N, const pstd_nop_gate* g, const pstd_nop_problem* prob, const float* p0,
                     const float* c0, float* out, int32_t batch, double tol, int32_t* fallback, int32_t* n_fallback) {
  if (!N || !g || !prob || !p0 || !c0 || !out) return fail(PSTD_E_INVALID_ARG, "null pointer");
  if (batch < 1) return fail(PSTD_E_INVALID_ARG, "batch < 1");
  if (!(tol >= 0) || !std::isfinite(tol)) return fail(PSTD_E_INVALID_ARG, "tol must be finite and >= 0");
  if (!(prob->dx > 0) || !(prob->dt > 0) || !(prob->rho0 > 0) || prob->steps < 0)
    return fail(PSTD_E_INVALID_ARG, "dx, dt, rho0 must be positive and steps >= 0");
  for (int f = 0; f < 4; ++f)
    if (prob->bc[f] != PSTD_NEUMANN && prob->bc[f] != PSTD_DIRICHLET)
      return fail(PSTD_E_INVALID_ARG, "the fallback solver takes Neumann or Dirichlet faces");
  if (g->wall_margin < 0) return fail(PSTD_E_INVALID_ARG, "wall_margin < 0");
  const int H = N->cfg.H, W = N->cfg.W, mb = N->cfg.max_batch;
  const int64_t P = N->P;
  // 1. input statistics, at most max_batch samples per call
  std::vector<double> st(4 * static_cast<size_t>(batch));
  for (int s0 = 0; s0 < batch; s0 += mb) {
    const int n = std::min(mb, batch - s0);
    const int r = pstd_nop_input_stats(N, p0 + s0 * P, c0 + s0 * P, n, g->wall_margin, st.data() + 4 * s0);
    if (r != PSTD_OK) return r;
  }
  // 2. the gate: inside the training distribution and a tolerance the validated error meets
  std::vector<int32_t> fb(batch);
  int32_t nf = 0;
  for (int b = 0; b < batch; ++b) {
    const double* x = st.data() + 4 * b;
    const bool inside = x[0] >= g->c0_lo && x[1] <= g->c0_hi && x[2] <= g->p_max && x[3] <= g->wall_share_max;
    fb[b] = (!inside || g->validated_error > tol) ? 1 : 0;
    nf += fb[b];
  }
  // 3. the surrogate on every chunk that holds an admitted sample (fallback rows are overwritten below)
  for (int s0 = 0; s0 < batch; s0 += mb) {
    const int n = std::min(mb, batch - s0);
    bool any = false;
    for (int b = s0; b < s0 + n; ++b) any = any || !fb[b];
    if (!any) continue;
    const int r = pstd_nop_infer(N, p0 + s0 * P, c0 + s0 * P, out + s0 * P, n);
    if (r != PSTD_OK) return r;
  }
  // 4. the FP32 batched solver for the rest: each such sample's pressure is stepped in place in out
  if (nf > 0) {
    std::vector<int64_t> nn(2 * static_cast<size_t>(nf));
    std::vector<int32_t> bc(4 * static_cast<size_t>(nf));
    std::vector<double> dx(nf, prob->dx), dt(nf, prob->dt), cmax(nf);
    std::vector<const float*> maps(nf);
    std::vector<pstd_state> states(nf);
    float* ubuf = nullptr;
    const int64_t ux = static_cast<int64_t>(H - 1) * W, uy = static_cast<int64_t>(H) * (W - 1);
    if (hipMalloc(&ubuf, sizeof(float) * (ux + uy) * nf) != hipSuccess)
      return fail(PSTD_E_OOM, "hipMalloc of the fallback velocities failed");
    int i = 0;
    int r = PSTD_OK;
    for (int b = 0; b < batch && r == PSTD_OK; ++b) {
      if (!fb[b]) continue;
      nn[2 * i] = H;
      nn[2 * i + 1] = W;
      for (int f = 0; f < 4; ++f) bc[4 * i + f] = prob->bc[f];
      cmax[i] = st[4 * b + 1];
      maps[i] = c0 + b * P;
      states[i] = pstd_state{};
      states[i].p = out + b * P;
      states[i].u[0] = ubuf + i * (ux + uy);
      states[i].u[1] = ubuf + i * (ux + uy) + ux;
      if (hipMemcpyAsync(out + b * P, p0 + b * P, sizeof(float) * P, hipMemcpyDeviceToDevice, N->stream) != hipSuccess)
        r = fail(PSTD_E_HIP, "copying the fallback inputs failed");
      ++i;
    }
    pstd_batch B = nullptr;
    if (r == PSTD_OK)
      r = pstd_batch_create(nf, nn.data(), bc.data(), dx.data(), dt.data(), cmax.data(), prob->rho0, N->stream, &B);
    if (r == PSTD_OK) r = pstd_batch_set_c0_maps(B, maps.data());
    if (r == PSTD_OK) r = pstd_batch_state_init(B, states.data(), 0);
    if (r == PSTD_OK) r = pstd_batch_step(B, states.data(), prob->steps);
    if (r == PSTD_OK) r = pstd_batch_synchronize(B);
    if (B) (void)pstd_batch_destroy(B);
    (void)hipStreamSynchronize(N->stream);
    (void)hipFree(ubuf);
    if (r != PSTD_OK) return r;
  }
  if (fallback) std::memcpy(fallback, fb.data(), sizeof(int32_t) * batch);
  if (n_fallback) *n_fallback = nf;
  return PSTD_OK;
}

int pstd_nop_destroy(pstd_nop N) {
  if (!N) return PSTD_OK;
  (void)(N->stream ? hipStreamSynchronize(N->stream) : hipDeviceSynchronize());
  nop_free(N);
  return PSTD_OK;
}

}  // extern "C"
