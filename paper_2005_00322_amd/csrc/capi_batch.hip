// libpstd C ABI, batched 2D solves: creation, initialisation, persistent stepping, pairing, autotuning.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>

#include "common.h"

struct pstd_batch_s {
  int count = 0;
  double rho0 = 1000.0;
  hipStream_t stream = nullptr;
  std::vector<int> nx, ny;
  std::vector<int> bc;                        // count x 4
  std::vector<double> dx, dt, c0;
  std::vector<void*> c2maps;                  // owned c0^2 maps (null for homogeneous solves)
  // shared unscaled FP32 operators, one per (n, case): G ((n-1) x n) and D (n x (n-1))
  struct Op {
    pstd::DevOperator G, D;
  };
  std::map<std::pair<int, int>, Op> ops;
  std::vector<pstd::BatchSolve> solves;       // host copy (pointers filled per state set)
  pstd::BatchSolve* d_solves = nullptr;
  std::vector<void*> key;                     // state pointers the device table was built for
  std::vector<pstd::BatchTask> tasksA, tasksB;
  int segA[pstd::kBatchQueues + 1] = {}, segB[pstd::kBatchQueues + 1] = {};   // queue boundaries
  pstd::BatchTask* d_tasks = nullptr;         // A then B
  int order_built = -1;
  int tile_built = -1;
  unsigned* d_counters = nullptr;             // kBatchCountersPerStep per step of a launch, then the timeout flag
  int blocks = 0;                             // 0 = occupancy maximum
  int order = 0;
  int tile = 32;                              // output tile edge of the persistent kernel (32 or 64)
  hipStream_t capture = nullptr;              // private stream the launch graphs are captured on
  std::map<std::tuple<int64_t, int, int>, hipGraphExec_t> graphs;   // (steps, blocks, tile) -> graph
};

namespace pstd {
namespace {

constexpr int64_t kChunk = 1024;   // steps per persistent launch

int upload_unscaled(const std::vector<double>& m, int M, int K, DevOperator* op) {
  op->M = M;
  op->K = K;
  op->Mp = static_cast<int>(round_up(M, kRowPad));
  op->Kp = static_cast<int>(round_up(K, kColPad));
  std::vector<float> h(static_cast<size_t>(op->Mp) * op->Kp, 0.f);
  for (int i = 0; i < M; ++i)
    for (int k = 0; k < K; ++k) h[static_cast<size_t>(i) * op->Kp + k] = static_cast<float>(m[static_cast<size_t>(i) * K + k]);
  if (hipMalloc(&op->data, h.size() * sizeof(float)) != hipSuccess) return fail(PSTD_E_OOM, "hipMalloc failed");
  PSTD_HIP(hipMemcpy(op->data, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
  return PSTD_OK;
}

void free_batch(pstd_batch_s* B) {
  if (!B) return;
  for (void* p : B->c2maps)
    if (p) (void)hipFree(p);
  for (auto& kv : B->ops) {
    if (kv.second.G.data) (void)hipFree(kv.second.G.data);
    if (kv.second.D.data) (void)hipFree(kv.second.D.data);
  }
  if (B->d_solves) (void)hipFree(B->d_solves);
  if (B->d_tasks) (void)hipFree(B->d_tasks);
  if (B->d_counters) (void)hipFree(B->d_counters);
  for (auto& kv : B->graphs) (void)hipGraphExecDestroy(kv.second);
  if (B->capture) (void)hipStreamDestroy(B->capture);
  delete B;
}

// Tile lists of both phases for output tiles of edge T, in the requested order.
// Tile lists of both phases, split into one queue per XCD.  Solves go to queues greedily, most costly
// first (cost: per-step multiply-adds, n_x n_y (n_x + n_y)), so each queue carries about 1/8 of the work
// and all tiles of a solve share one L2.  Within a queue: order 0 longest contraction first (stable, so
// a solve's tiles stay together), order 1 solve after solve.
void build_tasks(pstd_batch_s* B, int order, int T) {
  constexpr int Q = kBatchQueues;
  B->tasksA.clear();
  B->tasksB.clear();
  std::vector<int> by_cost(B->count);
  for (int s = 0; s < B->count; ++s) by_cost[s] = s;
  auto cost = [&](int s) { return static_cast<double>(B->nx[s]) * B->ny[s] * (B->nx[s] + B->ny[s]); };
  std::stable_sort(by_cost.begin(), by_cost.end(), [&](int x, int y) { return cost(x) > cost(y); });
  std::vector<double> load(Q, 0.0);
  std::vector<std::vector<int>> members(Q);
  for (int s : by_cost) {
    const int q = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
    members[q].push_back(s);
    load[q] += cost(s);
  }
  B->segA[0] = B->segB[0] = 0;
  for (int q = 0; q < Q; ++q) {
    std::sort(members[q].begin(), members[q].end());
    std::vector<std::pair<int, BatchTask>> a, b;   // (contracted length, task)
    for (int s : members[q]) {
      const int nx = B->nx[s], ny = B->ny[s];
      for (int i0 = 0; i0 < nx - 1; i0 += T)
        for (int j0 = 0; j0 < ny; j0 += T) a.push_back({nx, BatchTask{s, 0, i0, j0}});
      for (int i0 = 0; i0 < nx; i0 += T)
        for (int j0 = 0; j0 < ny - 1; j0 += T) a.push_back({ny, BatchTask{s, 1, i0, j0}});
      for (int i0 = 0; i0 < nx; i0 += T)
        for (int j0 = 0; j0 < ny; j0 += T) b.push_back({nx + ny - 2, BatchTask{s, 2, i0, j0}});
    }
    if (order == 0) {
      auto longest_first = [](const std::pair<int, BatchTask>& x, const std::pair<int, BatchTask>& y) {
        return x.first > y.first;
      };
      std::stable_sort(a.begin(), a.end(), longest_first);
      std::stable_sort(b.begin(), b.end(), longest_first);
    }
    for (auto& t : a) B->tasksA.push_back(t.second);
    for (auto& t : b) B->tasksB.push_back(t.second);
    B->segA[q + 1] = static_cast<int>(B->tasksA.size());
    B->segB[q + 1] = static_cast<int>(B->tasksB.size());
  }
}

int ensure_tasks(pstd_batch_s* B) {
  if (B->order_built == B->order && B->tile_built == B->tile && B->d_tasks) return PSTD_OK;
  if (!B->d_tasks) {
    // sized for the smallest tile (the longest lists); the address stays fixed for captured graphs
    build_tasks(B, 0, 32);
    const size_t n = B->tasksA.size() + B->tasksB.size();
    if (hipMalloc(&B->d_tasks, n * sizeof(BatchTask)) != hipSuccess)
      return fail(PSTD_E_OOM, "hipMalloc of the task lists failed");
  }
  build_tasks(B, B->order, B->tile);
  // the stream may still run a launch reading the previous lists
  PSTD_HIP(B->stream ? hipStreamSynchronize(B->stream) : hipDeviceSynchronize());
  PSTD_HIP(hipMemcpy(B->d_tasks, B->tasksA.data(), B->tasksA.size() * sizeof(BatchTask), hipMemcpyHostToDevice));
  PSTD_HIP(hipMemcpy(B->d_tasks + B->tasksA.size(), B->tasksB.data(), B->tasksB.size() * sizeof(BatchTask),
                     hipMemcpyHostToDevice));
  B->order_built = B->order;
  B->tile_built = B->tile;
  return PSTD_OK;
}

int ensure_solves(pstd_batch_s* B, const pstd_state* st) {
  std::vector<void*> key;
  for (int s = 0; s < B->count; ++s) {
    if (!st[s].p || !st[s].u[0] || !st[s].u[1]) return fail(PSTD_E_INVALID_ARG, "state %d has a null pointer", s);
    key.push_back(st[s].p);
    key.push_back(st[s].u[0]);
    key.push_back(st[s].u[1]);
  }
  if (key == B->key && B->d_solves) return PSTD_OK;
  for (int s = 0; s < B->count; ++s) {
    B->solves[s].p = static_cast<float*>(st[s].p);
    B->solves[s].ux = static_cast<float*>(st[s].u[0]);
    B->solves[s].uy = static_cast<float*>(st[s].u[1]);
  }
  if (!B->d_solves && hipMalloc(&B->d_solves, B->solves.size() * sizeof(BatchSolve)) != hipSuccess)
    return fail(PSTD_E_OOM, "hipMalloc of the solve table failed");
  // the stream may still run kernels reading the previous table
  PSTD_HIP(B->stream ? hipStreamSynchronize(B->stream) : hipDeviceSynchronize());
  PSTD_HIP(hipMemcpy(B->d_solves, B->solves.data(), B->solves.size() * sizeof(BatchSolve), hipMemcpyHostToDevice));
  B->key = key;
  return PSTD_OK;
}

int resident_blocks(const pstd_batch_s* B, int* out) {
  int maxb = 0;
  if (batch2d_max_blocks(B->tile, &maxb) != 0 || maxb < 1) return fail(PSTD_E_HIP, "occupancy query failed");
  *out = (B->blocks > 0 && B->blocks < maxb) ? B->blocks : maxb;
  return PSTD_OK;
}

// The instantiated graph (counter fill + persistent launch) for `steps` steps on `blocks` blocks.  The
// device tables it reads (solves, tasks, counters) keep their addresses for the batch's lifetime; their
// contents are refreshed in place.
int graph_for(pstd_batch_s* B, int64_t steps, int blocks, hipGraphExec_t* out) {
  const auto key = std::make_tuple(steps, blocks, B->tile);
  auto it = B->graphs.find(key);
  if (it != B->graphs.end()) {
    *out = it->second;
    return PSTD_OK;
  }
  if (!B->capture) PSTD_HIP(hipStreamCreateWithFlags(&B->capture, hipStreamNonBlocking));
  BatchArgs a;
  a.solves = B->d_solves;
  a.tasksA = B->d_tasks;
  a.tasksB = B->d_tasks + B->tasksA.size();
  for (int q = 0; q <= kBatchQueues; ++q) {
    a.segA[q] = B->segA[q];
    a.segB[q] = B->segB[q];
  }
  a.counters = B->d_counters;
  a.timeout = B->d_counters + kBatchCountersPerStep * kChunk;
  a.steps = steps;
  hipGraph_t g = nullptr;
  PSTD_HIP(hipStreamBeginCapture(B->capture, hipStreamCaptureModeThreadLocal));
  const hipError_t le = launch_batch2d(a, B->tile, blocks, B->capture);
  hipError_t e = hipStreamEndCapture(B->capture, &g);
  if (le != hipSuccess) e = le;
  hipGraphExec_t ex = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(PSTD_E_HIP, "capture of the persistent launch failed: %s", hipGetErrorString(e));
  B->graphs[key] = ex;
  *out = ex;
  return PSTD_OK;
}

// Tile 16: every solve has one shape of at most 512 x 512 nodes, so a step is two fused phase launches
// over all solves (block = (16 x 16 tile, solve)), as for a single 2D plan; no tasks, counters or grid
// barriers.  Graphs of up to kPhaseChunk steps are captured and replayed.
constexpr int64_t kPhaseChunk = 64;

bool phase_eligible(const pstd_batch_s* B) {
  if (B->count < 1 || B->count > 65535 || B->solves.size() != static_cast<size_t>(B->count)) return false;
  for (int s = 0; s < B->count; ++s) {
    const BatchSolve& S = B->solves[s];
    if (B->nx[s] != B->nx[0] || B->ny[s] != B->ny[0]) return false;
    if (!batch2d_phase_fits(S.ldgx, S.ldgy, S.lddx, S.lddy, S.nx, S.ny)) return false;
  }
  return phase2d_supported(B->nx[0], B->ny[0]);
}

int launch_phase_steps(pstd_batch_s* B, int64_t n_steps, hipStream_t s) {
  for (int64_t left = n_steps; left > 0; left -= kPhaseChunk) {
    const int64_t steps = std::min(left, kPhaseChunk);
    const auto key = std::make_tuple(steps, -1, 16);
    auto it = B->graphs.find(key);
    if (it == B->graphs.end()) {
      if (!B->capture) PSTD_HIP(hipStreamCreateWithFlags(&B->capture, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      PSTD_HIP(hipStreamBeginCapture(B->capture, hipStreamCaptureModeThreadLocal));
      hipError_t le = hipSuccess;
      for (int64_t k = 0; k < steps && le == hipSuccess; ++k) {
        le = launch_phase2d_batch(0, B->d_solves, B->count, B->nx[0], B->ny[0], B->capture);
        if (le == hipSuccess) le = launch_phase2d_batch(1, B->d_solves, B->count, B->nx[0], B->ny[0], B->capture);
      }
      hipError_t e = hipStreamEndCapture(B->capture, &g);
      if (le != hipSuccess) e = le;
      hipGraphExec_t ex = nullptr;
      if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (e != hipSuccess) return fail(PSTD_E_HIP, "capture of the phase launches failed: %s", hipGetErrorString(e));
      it = B->graphs.emplace(key, ex).first;
    }
    PSTD_HIP(hipGraphLaunch(it->second, s));
  }
  return PSTD_OK;
}

int launch_steps(pstd_batch_s* B, int64_t n_steps, hipStream_t s) {
  int blocks = 0;
  int st = resident_blocks(B, &blocks);
  if (st != PSTD_OK) return st;
  for (int64_t left = n_steps; left > 0; left -= kChunk) {
    hipGraphExec_t ex = nullptr;
    st = graph_for(B, std::min(left, kChunk), blocks, &ex);
    if (st != PSTD_OK) return st;
    PSTD_HIP(hipGraphLaunch(ex, s));
  }
  return PSTD_OK;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

std::string signature(const pstd_batch_s* B) {
  uint64_t h = 1469598103934665603ull;
  h = fnv1a(h, &B->count, sizeof(B->count));
  h = fnv1a(h, B->nx.data(), B->nx.size() * sizeof(int));
  h = fnv1a(h, B->ny.data(), B->ny.size() * sizeof(int));
  h = fnv1a(h, B->bc.data(), B->bc.size() * sizeof(int));
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    h = fnv1a(h, prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
  char buf[32];
  snprintf(buf, sizeof(buf), "%016llx", static_cast<unsigned long long>(h));
  return buf;
}

bool read_cache(const char* path, const std::string& sig, int* blocks, int* order, int* tile) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char buf[512] = {0};
  const size_t n = fread(buf, 1, sizeof(buf) - 1, f);
  fclose(f);
  buf[n] = 0;
  char s[64] = {0};
  int b = 0, o = 0, t = 0;
  const char* p = strstr(buf, "\"signature\"");
  if (!p || sscanf(p, "\"signature\": \"%63[0-9a-f]\"", s) != 1) return false;
  const char* pb = strstr(buf, "\"blocks\"");
  const char* po = strstr(buf, "\"order\"");
  const char* pt = strstr(buf, "\"tile\"");
  if (!pb || !po || !pt || sscanf(pb, "\"blocks\": %d", &b) != 1 || sscanf(po, "\"order\": %d", &o) != 1 ||
      sscanf(pt, "\"tile\": %d", &t) != 1 || b < 0 || o < 0 || o > 1 || (t != 16 && t != 32 && t != 64))
    return false;
  if (sig != s) return false;
  *blocks = b;
  *order = o;
  *tile = t;
  return true;
}

}  // namespace
}  // namespace pstd

using namespace pstd;

extern "C" {

int pstd_batch_create(int32_t count, const int64_t* n, const int32_t* bc, const double* dx, const double* dt,
                      const double* c0, double rho0, void* hip_stream, pstd_batch* out) {
  if (!out) return fail(PSTD_E_INVALID_ARG, "out is null");
  *out = nullptr;
  if (count < 1 || !n || !bc || !dx || !dt || !c0) return fail(PSTD_E_INVALID_ARG, "bad count or null array");
  if (!(rho0 > 0) || !std::isfinite(rho0)) return fail(PSTD_E_INVALID_ARG, "rho0 must be positive");
  pstd_batch_s* B = new pstd_batch_s();
  B->count = count;
  B->rho0 = rho0;
  B->stream = static_cast<hipStream_t>(hip_stream);
  for (int s = 0; s < count; ++s) {
    const int64_t nx = n[2 * s], ny = n[2 * s + 1];
    if (nx < 3 || ny < 3 || nx > 512 || ny > 512) {
      free_batch(B);
      return fail(PSTD_E_UNSUPPORTED, "solve %d: %lld x %lld nodes (need 3..512 per axis)", s, (long long)nx, (long long)ny);
    }
    for (int f = 0; f < 4; ++f)
      if (bc[4 * s + f] != PSTD_NEUMANN && bc[4 * s + f] != PSTD_DIRICHLET) {
        free_batch(B);
        return fail(PSTD_E_INVALID_ARG, "solve %d: bad boundary condition", s);
      }
    if (!(dx[s] > 0) || !(dt[s] > 0) || !(c0[s] > 0) || !std::isfinite(dx[s]) || !std::isfinite(dt[s]) ||
        !std::isfinite(c0[s])) {
      free_batch(B);
      return fail(PSTD_E_INVALID_ARG, "solve %d: dx, dt, c0 must be positive", s);
    }
    const AxisTables& tx = axis_tables(static_cast<int>(nx), axis_case(bc[4 * s], bc[4 * s + 1]));
    const AxisTables& ty = axis_tables(static_cast<int>(ny), axis_case(bc[4 * s + 2], bc[4 * s + 3]));
    const double kmax = std::sqrt(tx.kmax * tx.kmax + ty.kmax * ty.kmax) / dx[s];
    if (c0[s] * dt[s] * kmax / 2.0 > 1.0) {
      free_batch(B);
      return fail(PSTD_E_UNSTABLE, "solve %d: c0*dt/dx = %g above the limit", s, c0[s] * dt[s] / dx[s]);
    }
    B->nx.push_back(static_cast<int>(nx));
    B->ny.push_back(static_cast<int>(ny));
    for (int f = 0; f < 4; ++f) B->bc.push_back(bc[4 * s + f]);
    B->dx.push_back(dx[s]);
    B->dt.push_back(dt[s]);
    B->c0.push_back(c0[s]);
  }
  // shared operators
  for (int s = 0; s < count; ++s) {
    const std::pair<int, int> keys[2] = {{B->nx[s], static_cast<int>(axis_case(B->bc[4 * s], B->bc[4 * s + 1]))},
                                         {B->ny[s], static_cast<int>(axis_case(B->bc[4 * s + 2], B->bc[4 * s + 3]))}};
    for (const auto& k : keys) {
      if (B->ops.count(k)) continue;
      const AxisTables& t = axis_tables(k.first, static_cast<AxisCase>(k.second));
      pstd_batch_s::Op op;
      int st = upload_unscaled(t.G, k.first - 1, k.first, &op.G);
      if (st == PSTD_OK) st = upload_unscaled(t.D, k.first, k.first - 1, &op.D);
      B->ops[k] = op;
      if (st != PSTD_OK) {
        free_batch(B);
        return st;
      }
    }
    const pstd_batch_s::Op& ox = B->ops[keys[0]];
    const pstd_batch_s::Op& oy = B->ops[keys[1]];
    BatchSolve S{};
    S.Gx = static_cast<const float*>(ox.G.data);
    S.Dx = static_cast<const float*>(ox.D.data);
    S.Gy = static_cast<const float*>(oy.G.data);
    S.Dy = static_cast<const float*>(oy.D.data);
    S.ldgx = ox.G.Kp;
    S.lddx = ox.D.Kp;
    S.ldgy = oy.G.Kp;
    S.lddy = oy.D.Kp;
    S.mgx = ox.G.Mp;
    S.mdx = ox.D.Mp;
    S.mgy = oy.G.Mp;
    S.mdy = oy.D.Mp;
    S.nx = B->nx[s];
    S.ny = B->ny[s];
    S.sG = -B->dt[s] / (rho0 * B->dx[s]);
    S.sD = -B->dt[s] * rho0 * B->c0[s] * B->c0[s] / B->dx[s];
    B->solves.push_back(S);
  }
  if (hipMalloc(&B->d_counters, sizeof(unsigned) * (kBatchCountersPerStep * kChunk + 1)) != hipSuccess) {
    free_batch(B);
    return fail(PSTD_E_OOM, "hipMalloc of the phase counters failed");
  }
  if (hipMemset(B->d_counters, 0, sizeof(unsigned) * (kBatchCountersPerStep * kChunk + 1)) != hipSuccess) {
    free_batch(B);
    return fail(PSTD_E_HIP, "hipMemset of the phase counters failed");
  }
  *out = B;
  return PSTD_OK;
}

int pstd_batch_set_c0_maps(pstd_batch B, const float* const* c0_maps) {
  if (!B || !c0_maps) return fail(PSTD_E_INVALID_ARG, "null batch or map array");
  B->c2maps.resize(B->count, nullptr);
  for (int s = 0; s < B->count; ++s) {
    if (!c0_maps[s]) continue;
    const int64_t np = static_cast<int64_t>(B->nx[s]) * B->ny[s];
    if (!B->c2maps[s] && hipMalloc(&B->c2maps[s], np * sizeof(float)) != hipSuccess)
      return fail(PSTD_E_OOM, "hipMalloc of a c0^2 map failed");
    PSTD_HIP(launch_square(PSTD_FP32, c0_maps[s], B->c2maps[s], np, B->stream));
    B->solves[s].c2 = static_cast<const float*>(B->c2maps[s]);
    B->solves[s].sD = -B->dt[s] * B->rho0 / B->dx[s];
  }
  B->key.clear();   // the device solve table is rebuilt with the maps on the next step
  return PSTD_OK;
}

int pstd_batch_synchronize(pstd_batch B) {
  if (!B) return fail(PSTD_E_INVALID_ARG, "null batch");
  PSTD_HIP(B->stream ? hipStreamSynchronize(B->stream) : hipDeviceSynchronize());
  unsigned flag = 0;
  PSTD_HIP(hipMemcpy(&flag, B->d_counters + kBatchCountersPerStep * kChunk, sizeof(unsigned), hipMemcpyDeviceToHost));
  if (flag) {
    PSTD_HIP(hipMemset(B->d_counters + kBatchCountersPerStep * kChunk, 0, sizeof(unsigned)));
    return fail(PSTD_E_HIP, "a grid barrier of the persistent launch timed out (blocks not all resident); "
                            "the state is not valid");
  }
  return PSTD_OK;
}

int pstd_batch_destroy(pstd_batch B) {
  if (!B) return PSTD_OK;
  (void)(B->stream ? hipStreamSynchronize(B->stream) : hipDeviceSynchronize());
  free_batch(B);
  return PSTD_OK;
}

int pstd_batch_state_init(pstd_batch B, pstd_state* st, int32_t u_mode) {
  if (!B || !st) return fail(PSTD_E_INVALID_ARG, "null batch or states");
  if (u_mode < 0 || u_mode > 2) return fail(PSTD_E_INVALID_ARG, "u_mode must be 0, 1 or 2");
  for (int s = 0; s < B->count; ++s) {
    if (!st[s].p || !st[s].u[0] || !st[s].u[1]) return fail(PSTD_E_INVALID_ARG, "state %d has a null pointer", s);
    const int64_t n[3] = {B->nx[s], B->ny[s], 1};
    const int lo[3] = {B->bc[4 * s] == PSTD_DIRICHLET, B->bc[4 * s + 2] == PSTD_DIRICHLET, 0};
    const int hi[3] = {B->bc[4 * s + 1] == PSTD_DIRICHLET, B->bc[4 * s + 3] == PSTD_DIRICHLET, 0};
    PSTD_HIP(launch_zero_dirichlet(PSTD_FP32, st[s].p, 2, n, lo, hi, B->stream));
    st[s].step = 0;
    if (u_mode == 2) continue;
    const BatchSolve& S = B->solves[s];
    for (int a = 0; a < 2; ++a) {
      const int64_t ucount = (a == 0 ? (S.nx - 1) * static_cast<int64_t>(S.ny) : S.nx * static_cast<int64_t>(S.ny - 1));
      if (u_mode == 1) {
        PSTD_HIP(launch_fill_zero(PSTD_FP32, st[s].u[a], ucount, B->stream));
        continue;
      }
      // u^{-1/2} = +(dt / (2 rho0)) G p = -1/2 sG (unscaled G) p
      ContractArgs c{};
      c.A = a == 0 ? S.Gx : S.Gy;
      c.lda = a == 0 ? S.ldgx : S.ldgy;
      c.M = (a == 0 ? S.nx : S.ny) - 1;
      c.K = a == 0 ? S.nx : S.ny;
      c.X = st[s].p;
      c.Y = st[s].u[a];
      c.alpha = static_cast<float>(-0.5 * S.sG);
      c.alpha_d = -0.5 * S.sG;
      c.beta = 0.f;
      c.beta_d = 0.0;
      c.scale = nullptr;
      if (a == 0) {
        c.ncols = S.ny;
        c.batch = 1;
        c.x_bstride = 0;
        c.y_bstride = 0;
      } else {
        c.ncols = S.nx;
        c.batch = 1;
        c.x_bstride = 0;
        c.y_bstride = 0;
      }
      PSTD_HIP(launch_contract_fp32(c, a == 1, B->stream));
    }
  }
  return PSTD_OK;
}

int pstd_batch_step(pstd_batch B, pstd_state* st, int64_t n_steps) {
  if (!B || !st) return fail(PSTD_E_INVALID_ARG, "null batch or states");
  if (n_steps < 0) return fail(PSTD_E_INVALID_ARG, "n_steps < 0");
  if (n_steps == 0) return PSTD_OK;
  int r = ensure_solves(B, st);
  if (B->tile == 16) {
    if (r == PSTD_OK) r = launch_phase_steps(B, n_steps, B->stream);
  } else {
    if (r == PSTD_OK) r = ensure_tasks(B);
    if (r == PSTD_OK) r = launch_steps(B, n_steps, B->stream);
  }
  if (r != PSTD_OK) return r;
  for (int s = 0; s < B->count; ++s) st[s].step += n_steps;
  return PSTD_OK;
}

int pstd_batch_combine_R(pstd_batch B, const pstd_state* st, const int32_t* pairs, const double* R, float* const* out,
                         int32_t npairs) {
  if (!B || !st || !pairs || !R || !out || npairs < 0) return fail(PSTD_E_INVALID_ARG, "null argument");
  for (int i = 0; i < npairs; ++i) {
    const int d = pairs[2 * i], nn = pairs[2 * i + 1];
    if (d < 0 || d >= B->count || nn < 0 || nn >= B->count) return fail(PSTD_E_INVALID_ARG, "pair %d out of range", i);
    if (B->nx[d] != B->nx[nn] || B->ny[d] != B->ny[nn]) return fail(PSTD_E_INVALID_ARG, "pair %d: sizes differ", i);
    if (!out[i] || !st[d].p || !st[nn].p || !std::isfinite(R[i])) return fail(PSTD_E_INVALID_ARG, "pair %d: bad argument", i);
    const float* f[2] = {static_cast<const float*>(st[nn].p), static_cast<const float*>(st[d].p)};
    const float w[2] = {static_cast<float>(0.5 * (1.0 + R[i])), static_cast<float>(0.5 * (1.0 - R[i]))};
    PSTD_HIP(launch_combine(f, w, 2, out[i], static_cast<int64_t>(B->nx[d]) * B->ny[d], B->stream));
  }
  return PSTD_OK;
}

int pstd_batch_set_config(pstd_batch B, int32_t blocks, int32_t order, int32_t tile) {
  if (!B || blocks < 0 || order < 0 || order > 1 || (tile != 16 && tile != 32 && tile != 64))
    return fail(PSTD_E_INVALID_ARG, "bad batch configuration");
  if (tile == 16 && !phase_eligible(B))
    return fail(PSTD_E_UNSUPPORTED, "tile 16 (fused phase launches) needs solves of one shape of at most 512 x 512");
  B->blocks = blocks;
  B->order = order;
  B->tile = tile;
  return PSTD_OK;
}

int pstd_batch_autotune(pstd_batch B, int32_t trial_steps, const char* cache_path, int32_t* config_out) {
  if (!B || trial_steps < 1) return fail(PSTD_E_INVALID_ARG, "bad batch or trial_steps");
  const std::string sig = signature(B);
  int cb = 0, co = 0, ct = 32;
  // a cached tile-16 entry is reused only where the fused phase launches apply (one shape of at most 512^2)
  if (cache_path && read_cache(cache_path, sig, &cb, &co, &ct) && (ct != 16 || phase_eligible(B))) {
    B->blocks = cb;
    B->order = co;
    B->tile = ct;
    if (config_out) {
      config_out[0] = cb;
      config_out[1] = co;
      config_out[2] = ct;
      config_out[3] = 1;
    }
    return PSTD_OK;
  }
  // scratch states (zero fields: the timing does not depend on the values)
  std::vector<pstd_state> scratch(B->count);
  std::vector<void*> bufs;
  int st = PSTD_OK;
  for (int s = 0; s < B->count && st == PSTD_OK; ++s) {
    const size_t np = static_cast<size_t>(B->nx[s]) * B->ny[s];
    const size_t nux = static_cast<size_t>(B->nx[s] - 1) * B->ny[s];
    const size_t nuy = static_cast<size_t>(B->nx[s]) * (B->ny[s] - 1);
    void* p[3] = {nullptr, nullptr, nullptr};
    const size_t sz[3] = {np, nux, nuy};
    for (int i = 0; i < 3; ++i) {
      if (hipMalloc(&p[i], sz[i] * sizeof(float)) != hipSuccess) {
        st = fail(PSTD_E_OOM, "autotune scratch allocation failed");
        break;
      }
      bufs.push_back(p[i]);
      if (launch_fill_zero(PSTD_FP32, p[i], static_cast<int64_t>(sz[i]), B->stream) != hipSuccess)
        st = fail(PSTD_E_HIP, "zero fill failed");
    }
    scratch[s].p = p[0];
    scratch[s].u[0] = p[1];
    scratch[s].u[1] = p[2];
    scratch[s].u[2] = nullptr;
    scratch[s].step = 0;
  }
  int cus = 0, dev = 0;
  if (st == PSTD_OK && (hipGetDevice(&dev) != hipSuccess ||
                        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess))
    st = fail(PSTD_E_HIP, "device query failed");
  const std::vector<void*> saved_key = B->key;
  double best = 1e300;
  int best_b = 0, best_o = 0, best_t = 32;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (st == PSTD_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    st = fail(PSTD_E_HIP, "event creation failed");
  if (st == PSTD_OK && phase_eligible(B)) {
    // the fused phase launches: one configuration
    B->tile = 16;
    B->blocks = 0;
    B->order = 0;
    st = ensure_solves(B, scratch.data());
    if (st == PSTD_OK) st = launch_phase_steps(B, trial_steps, B->stream);   // warm (and capture the graph)
    if (st == PSTD_OK && hipEventRecord(e0, B->stream) != hipSuccess) st = fail(PSTD_E_HIP, "event record failed");
    if (st == PSTD_OK) st = launch_phase_steps(B, trial_steps, B->stream);
    if (st == PSTD_OK && (hipEventRecord(e1, B->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
      st = fail(PSTD_E_HIP, "event timing failed");
    if (st == PSTD_OK) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      best = ms;
      best_b = 0;
      best_o = 0;
      best_t = 16;
    }
  }
  for (int tile : {32, 64}) {
    if (st != PSTD_OK) break;
    int maxb = 0;
    if (batch2d_max_blocks(tile, &maxb) != 0 || maxb < 1) {
      st = fail(PSTD_E_HIP, "occupancy query failed");
      break;
    }
    std::vector<int> cand;
    for (int m = 1; m * cus <= maxb; ++m) cand.push_back(m * cus);
    if (cand.empty() || cand.back() != maxb) cand.push_back(maxb);
    for (int order = 0; order < 2 && st == PSTD_OK; ++order)
      for (int b : cand) {
        B->blocks = b == maxb ? 0 : b;
        B->order = order;
        B->tile = tile;
        st = ensure_solves(B, scratch.data());
        if (st == PSTD_OK) st = ensure_tasks(B);
        if (st == PSTD_OK) st = launch_steps(B, trial_steps, B->stream);   // warm (and capture the graph)
        if (st != PSTD_OK) break;
        if (hipEventRecord(e0, B->stream) != hipSuccess) { st = fail(PSTD_E_HIP, "event record failed"); break; }
        st = launch_steps(B, trial_steps, B->stream);
        if (st != PSTD_OK) break;
        if (hipEventRecord(e1, B->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          st = fail(PSTD_E_HIP, "event timing failed");
          break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
          best = ms;
          best_b = B->blocks;
          best_o = order;
          best_t = tile;
        }
      }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)(B->stream ? hipStreamSynchronize(B->stream) : hipDeviceSynchronize());
  for (void* p : bufs) (void)hipFree(p);
  B->key.clear();   // the device solve table points at the freed scratch states
  (void)saved_key;
  if (st != PSTD_OK) return st;
  B->blocks = best_b;
  B->order = best_o;
  B->tile = best_t;
  if (cache_path) {
    FILE* f = fopen(cache_path, "w");
    if (f) {
      fprintf(f, "{\"signature\": \"%s\", \"blocks\": %d, \"order\": %d, \"tile\": %d, \"ms_per_step\": %.6f}\n",
              sig.c_str(), B->blocks, B->order, B->tile, best / trial_steps);
      fclose(f);
    }
  }
  if (config_out) {
    config_out[0] = B->blocks;
    config_out[1] = B->order;
    config_out[2] = B->tile;
    config_out[3] = 0;
  }
  return PSTD_OK;
}

}  // extern "C"
