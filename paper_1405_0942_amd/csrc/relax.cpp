// relax.cpp -- C ABI of the relaxation library (include/relax.h): configuration checks,
// workspace carving, the launch sequence of a Cash-Karp step and the host side of the
// device step controller.
#include "relax.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "relax_device.h"

using namespace relax;

namespace {

constexpr size_t ALIGN = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }
constexpr size_t STAGGER = 65536 + ALIGN;

struct Layout {
  size_t ctl, x0, x1, k[3], y3, d4, y5, sum[3], B0, B0_64, part, lam, ring, out, dtrec, ckpt, total;
  // reverse mode (record = 1): segment positions and stage vectors, cotangents, seed
  size_t ctl2, seg_x, seg_k, seg_y, Fbar, xbar, ybar, ubar, B0bar, useed;
  int ckpt_slots;
};

struct Ctx {
  relax_config cfg;
  int K_record = 0;
  Geometry g{};
  hipStream_t stream = nullptr;
  bool mixed = false;
  char* base = nullptr;
  Layout L{};
  Control* d_ctl = nullptr;
  double* d_x[2] = {nullptr, nullptr};
  void* d_k[3] = {};
  void* d_sum[3] = {};
  void* d_d4 = nullptr;
  double* d_y3 = nullptr;
  double* d_y5 = nullptr;
  void* d_B0 = nullptr;
  double* d_B0_64 = nullptr;
  double* d_part = nullptr;
  double* d_lam = nullptr;
  double* d_ring = nullptr;
  double* d_out = nullptr;
  double* d_dtrec = nullptr;
  double* d_ckpt = nullptr;
  Control* d_ctl2 = nullptr;
  double* d_seg_x = nullptr;
  double* d_seg_k = nullptr;
  double* d_seg_y = nullptr;
  double* d_ubar = nullptr;
  double* d_Fbar = nullptr;
  double* d_xbar = nullptr;
  double* d_ybar = nullptr;
  double* d_B0bar = nullptr;
  double* d_useed = nullptr;
  Control* h_ctl = nullptr;  // pinned mirror of the control block
  double* h_ring = nullptr;  // pinned copy of the diagnostics ring
  int status = RELAX_OK;
  int cur = 0;  // host mirror of ctl->cur, valid between calls
  std::string err;
  // optional per-kernel timing (relax_profile)
  bool profiling = false;
  std::vector<hipEvent_t> ev;       // event pool, pairs per launch
  std::vector<int> ev_kind;         // kernel kind of each recorded pair
  size_t ev_used = 0;               // pairs recorded since the last harvest
  double prof_ms[8] = {0};          // accumulated ms per kind: stages 1..6 -> 0..5, control -> 6
  long long prof_n[8] = {0};
};

int fail(Ctx* c, int code, const std::string& msg) {
  if (c) {
    c->err = msg;
    if (code == RELAX_E_FOLD || code == RELAX_E_DT || code == RELAX_E_NAN || code == RELAX_E_HIP) c->status = code;
  }
  return code;
}

#define HIP_TRY(ctx, expr)                                                             \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail((ctx), RELAX_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

// configuration checks and the sweep geometry (also used by noalloc.hip)
namespace relax {

bool valid_config(const relax_config* c) {
  if (!c) return false;
  for (int a = 0; a < 3; a++) {
    if (c->n[a] < 4 || !(c->h[a] > 0.0) || !std::isfinite(c->h[a])) return false;
    if (c->bc[a] != RELAX_LINE_TIED && c->bc[a] != RELAX_PERIODIC) return false;
  }
  if ((long long)c->n[0] * c->n[1] >= (1LL << 28) || (long long)c->n[0] * c->n[1] * c->n[2] > (1LL << 40)) return false;
  if (c->precision != RELAX_FP64 && c->precision != RELAX_FP32_MIXED) return false;
  if (!std::isfinite(c->gamma) || !(c->dt0 > 0.0) || !std::isfinite(c->dt0)) return false;
  if (!(c->dt_min >= 0.0) || !(c->tol > 0.0) || !(c->xi_null_tau >= 0.0)) return false;
  if (!(c->safety > 0.0 && c->safety <= 1.0)) return false;
  if (c->adaptive != 0 && c->adaptive != 1) return false;
  if (c->record != 0 && c->record != 1) return false;
  if (c->record && c->checkpoint_every < 1) return false;
  if (c->curl != RELAX_CURL_NN && c->curl != RELAX_CURL_NNN) return false;
  if (c->curl == RELAX_CURL_NNN && c->precision != RELAX_FP64) return false;
  return true;
}

// z-chunk length.  A sweep's workgroups march their chunks concurrently, one resident per CU
// on 256 CUs (256 slots: 91 KB of LDS in FP64, and the mixed sweeps' registers leave room for
// one 8-wave workgroup), so a sweep takes about ceil(workgroups / 256) rounds, each as long as
// one chunk: tz planes plus the ~4 planes a chunk loads before its first output.  The chunk
// count minimises rounds x (tz + 4) with tz >= 8 (the fewer chunks on a tie): a grid whose
// x-y tiles alone slightly exceed the slots would otherwise run a second, nearly empty round
// as long as the first, and a small grid would leave most CUs idle.
int choose_tz(const relax_config* c, int tiles_xy) {
  if (const char* e = std::getenv("RELAX_TZ")) {
    int v = std::atoi(e);
    if (v >= 1) return std::min(v, c->n[2]);
  }
  const long long slots = 256;
  const int nz = c->n[2];
  int best_tz = nz;
  long long best_cost = -1;
  for (int chunks = 1; chunks <= std::max(1, nz / 8); chunks++) {
    const int tz = (nz + chunks - 1) / chunks;
    const long long blocks = (long long)tiles_xy * ((nz + tz - 1) / tz);
    const long long cost = ((blocks + slots - 1) / slots) * (tz + 4);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best_tz = tz;
    }
  }
  return best_tz;
}

Geometry make_geometry(const relax_config* c) {
  Geometry g{};
  for (int a = 0; a < 3; a++) {
    g.n[a] = c->n[a];
    g.bc[a] = c->bc[a];
    g.h[a] = c->h[a];
    g.period[a] = c->n[a] * c->h[a];
  }
  g.N = (long long)c->n[0] * c->n[1] * c->n[2];
  g.dV = c->h[0] * c->h[1] * c->h[2];
  g.inv8h3 = 1.0 / (8.0 * c->h[0] * c->h[1] * c->h[2]);
  g.b0scale[0] = 4.0 * c->h[1] * c->h[2];
  g.b0scale[1] = 4.0 * c->h[2] * c->h[0];
  g.b0scale[2] = 4.0 * c->h[0] * c->h[1];
  g.tiles[0] = (c->n[0] + TX - 1) / TX;
  g.tiles[1] = (c->n[1] + TY - 1) / TY;
  g.tz = choose_tz(c, g.tiles[0] * g.tiles[1]);
  g.tiles[2] = (c->n[2] + g.tz - 1) / g.tz;
  g.nblocks = g.tiles[0] * g.tiles[1] * g.tiles[2];
  g.curl = c->curl;
  return g;
}

}  // namespace relax

namespace {

Layout make_layout(const relax_config* c, const Geometry& g, int K_record) {
  Layout L{};
  const size_t N3 = 3 * (size_t)g.N;
  const size_t ts = (c->precision == RELAX_FP32_MIXED) ? sizeof(float) : sizeof(double);
  size_t off = 0;
  // consecutive arrays start STAGGER bytes further apart than their sizes: on power-of-two
  // grids the arrays would otherwise be exact multiples of 2^k bytes apart, and the same node
  // of every array the sweeps stream at once would fall on the same memory channel
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes) + STAGGER;
    return o;
  };
  L.ctl = take(sizeof(Control));
  L.x0 = take(N3 * sizeof(double));
  L.x1 = take(N3 * sizeof(double));
  // k_1..k_3, the stage inputs y_3 and y_5 (FP64), the stage-4 increment d_4 and the partial
  // sums P6, X, E (stage.hip)
  for (int s = 0; s < 3; s++) L.k[s] = take(N3 * ts);
  L.y3 = take(N3 * sizeof(double));
  L.d4 = take(N3 * ts);
  L.y5 = take(N3 * sizeof(double));
  for (int i = 0; i < 3; i++) L.sum[i] = take(N3 * ts);
  L.B0_64 = take(N3 * sizeof(double));
  L.B0 = (c->precision == RELAX_FP32_MIXED) ? take(N3 * sizeof(float)) : L.B0_64;
  L.part = take((size_t)g.nblocks * NPART * sizeof(double));
  L.lam = take((size_t)g.nblocks * sizeof(double));
  L.ring = take((size_t)RING_CAP * 8 * sizeof(double));
  L.out = take(16 * sizeof(double));
  L.ckpt_slots = 0;
  L.dtrec = L.ckpt = 0;
  L.ctl2 = L.seg_x = L.seg_k = L.seg_y = L.Fbar = L.xbar = L.ybar = L.ubar = L.B0bar = L.useed = 0;
  if (c->record && K_record > 0) {
    const size_t cpe = (size_t)c->checkpoint_every;
    L.dtrec = take((size_t)K_record * sizeof(double));
    L.ckpt_slots = K_record / c->checkpoint_every + 1;
    L.ckpt = take((size_t)L.ckpt_slots * N3 * sizeof(double));
    L.ctl2 = take(sizeof(Control));
    L.seg_x = take((cpe + 1) * N3 * sizeof(double));
    L.seg_k = take(cpe * 3 * N3 * sizeof(double));
    L.seg_y = take(cpe * 4 * N3 * sizeof(double));
    L.Fbar = take(3 * N3 * sizeof(double));
    L.xbar = take(N3 * sizeof(double));
    L.ybar = take(5 * N3 * sizeof(double));
    L.ubar = take(N3 * sizeof(double));
    L.B0bar = take(N3 * sizeof(double));
    L.useed = take(N3 * sizeof(double));
  }
  L.total = off;
  return L;
}

int sync_ctl(Ctx* c) {
  HIP_TRY(c, hipMemcpyAsync(c->h_ctl, c->d_ctl, sizeof(Control), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->cur = c->h_ctl->cur;
  return RELAX_OK;
}

int push_ctl(Ctx* c) {
  HIP_TRY(c, hipMemcpyAsync(c->d_ctl, c->h_ctl, sizeof(Control), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return RELAX_OK;
}

SweepArgs sweep_args(Ctx* c) {
  SweepArgs a{};
  a.g = c->g;
  a.x[0] = c->d_x[0];
  a.x[1] = c->d_x[1];
  a.xout[0] = c->d_x[0];
  a.xout[1] = c->d_x[1];
  for (int s = 0; s < 3; s++) a.k[s] = c->d_k[s];
  a.y3 = c->d_y3;
  a.d4 = c->d_d4;
  a.y5 = c->d_y5;
  for (int i = 0; i < 3; i++) a.sum[i] = c->d_sum[i];
  a.yrec[0] = a.yrec[1] = nullptr;
  a.B0 = c->d_B0;
  a.ctl = c->d_ctl;
  a.part = c->d_part;
  a.lam_part = c->d_lam;
  a.ckpt = c->d_ckpt;
  a.ckpt_slots = c->L.ckpt_slots;
  a.diag_buf = 0;
  a.u_out = nullptr;
  a.u_det_scale = 0.0;
  a.b0_mul[0] = a.b0_mul[1] = a.b0_mul[2] = 1.0;
  return a;
}

// FP64 diagnostics sweep of x[buf] into d_out[0..5] = {E, R2, xi, min det, nulls, concave}; host copy.
// Non-null u_out, B_out, J_out, alpha_out, kappa_out also receive u, B, J, alpha* and the
// convexity of x[buf].
int diagnostics_sweep(Ctx* c, int buf, double out[6], double* u_out = nullptr, double u_det_scale = 0.0,
                      double* B_out = nullptr, double* J_out = nullptr, double* alpha_out = nullptr,
                      int* kappa_out = nullptr) {
  SweepArgs a = sweep_args(c);
  a.B0 = c->d_B0_64;
  a.diag_buf = buf;
  a.u_out = u_out;
  a.u_det_scale = u_det_scale;
  a.B_out = B_out;
  a.J_out = J_out;
  a.alpha_out = alpha_out;
  a.kappa_out = kappa_out;
  HIP_TRY(c, launch_diagnostics(a, c->stream));
  HIP_TRY(c, launch_diag_finish(c->d_part, c->g.nblocks, c->g.dV, c->d_out, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->h_ring, c->d_out, 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::memcpy(out, c->h_ring, 6 * sizeof(double));
  return RELAX_OK;
}

// profiling: event pair around one launch of kernel kind `kind`
int prof_begin(Ctx* c, int kind) {
  if (c->ev_used * 2 + 2 > c->ev.size()) {
    for (int i = 0; i < 2; i++) {
      hipEvent_t e;
      HIP_TRY(c, hipEventCreate(&e));
      c->ev.push_back(e);
    }
  }
  if (c->ev_kind.size() <= c->ev_used) c->ev_kind.resize(c->ev_used + 1);
  c->ev_kind[c->ev_used] = kind;
  HIP_TRY(c, hipEventRecord(c->ev[2 * c->ev_used], c->stream));
  return RELAX_OK;
}

int prof_end(Ctx* c) {
  HIP_TRY(c, hipEventRecord(c->ev[2 * c->ev_used + 1], c->stream));
  c->ev_used++;
  return RELAX_OK;
}

// after a stream synchronisation: add the recorded pairs to the totals
int prof_harvest(Ctx* c) {
  for (size_t i = 0; i < c->ev_used; i++) {
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
    c->prof_ms[c->ev_kind[i]] += ms;
    c->prof_n[c->ev_kind[i]] += 1;
  }
  c->ev_used = 0;
  return RELAX_OK;
}

int enqueue_attempts(Ctx* c, int count) {
  const SweepArgs a = sweep_args(c);
  int rc;
  for (int i = 0; i < count; i++) {
    for (int s = 1; s <= 6; s++) {
      if (c->profiling && (rc = prof_begin(c, s - 1))) return rc;
      HIP_TRY(c, launch_stage(s, c->mixed, a, c->stream));
      if (c->profiling && (rc = prof_end(c))) return rc;
    }
    if (c->profiling && (rc = prof_begin(c, 6))) return rc;
    HIP_TRY(c, launch_control(c->d_ctl, c->d_part, c->d_lam, c->g.nblocks, c->d_ring, c->d_dtrec, c->stream));
    if (c->profiling && (rc = prof_end(c))) return rc;
  }
  return RELAX_OK;
}

}  // namespace

extern "C" {

size_t relax_workspace_bytes(const relax_config* cfg, int K_record) {
  if (!valid_config(cfg) || K_record < 0) return 0;
  Geometry g = make_geometry(cfg);
  return make_layout(cfg, g, cfg->record ? K_record : 0).total;
}

int relax_init(const relax_config* cfg, int K_record, const double* d_x0, const double* d_B0, void* d_workspace,
               size_t workspace_bytes, void* hip_stream, void** out_ctx) {
  if (!out_ctx) return RELAX_E_ARG;
  *out_ctx = nullptr;
  if (!valid_config(cfg) || K_record < 0 || !d_x0 || !d_B0 || !d_workspace) return RELAX_E_ARG;
  if (reinterpret_cast<uintptr_t>(d_workspace) % ALIGN != 0) return RELAX_E_ARG;
  Ctx* c = new (std::nothrow) Ctx();
  if (!c) return RELAX_E_ARG;
  c->cfg = *cfg;
  c->K_record = cfg->record ? K_record : 0;
  c->g = make_geometry(cfg);
  c->L = make_layout(cfg, c->g, c->K_record);
  if (workspace_bytes < c->L.total) {
    delete c;
    return RELAX_E_SPACE;
  }
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->mixed = (cfg->precision == RELAX_FP32_MIXED);
  c->base = static_cast<char*>(d_workspace);
  const Layout& L = c->L;
  c->d_ctl = reinterpret_cast<Control*>(c->base + L.ctl);
  c->d_x[0] = reinterpret_cast<double*>(c->base + L.x0);
  c->d_x[1] = reinterpret_cast<double*>(c->base + L.x1);
  for (int s = 0; s < 3; s++) c->d_k[s] = c->base + L.k[s];
  c->d_y3 = reinterpret_cast<double*>(c->base + L.y3);
  c->d_d4 = c->base + L.d4;
  c->d_y5 = reinterpret_cast<double*>(c->base + L.y5);
  for (int i = 0; i < 3; i++) c->d_sum[i] = c->base + L.sum[i];
  c->d_B0_64 = reinterpret_cast<double*>(c->base + L.B0_64);
  c->d_B0 = c->base + L.B0;
  c->d_part = reinterpret_cast<double*>(c->base + L.part);
  c->d_lam = reinterpret_cast<double*>(c->base + L.lam);
  c->d_ring = reinterpret_cast<double*>(c->base + L.ring);
  c->d_out = reinterpret_cast<double*>(c->base + L.out);
  if (L.ckpt_slots > 0) {
    c->d_dtrec = reinterpret_cast<double*>(c->base + L.dtrec);
    c->d_ckpt = reinterpret_cast<double*>(c->base + L.ckpt);
    c->d_ctl2 = reinterpret_cast<Control*>(c->base + L.ctl2);
    c->d_seg_x = reinterpret_cast<double*>(c->base + L.seg_x);
    c->d_seg_k = reinterpret_cast<double*>(c->base + L.seg_k);
    c->d_seg_y = reinterpret_cast<double*>(c->base + L.seg_y);
    c->d_ubar = reinterpret_cast<double*>(c->base + L.ubar);
    c->d_Fbar = reinterpret_cast<double*>(c->base + L.Fbar);
    c->d_xbar = reinterpret_cast<double*>(c->base + L.xbar);
    c->d_ybar = reinterpret_cast<double*>(c->base + L.ybar);
    c->d_B0bar = reinterpret_cast<double*>(c->base + L.B0bar);
    c->d_useed = reinterpret_cast<double*>(c->base + L.useed);
  }
  int rc = RELAX_OK;
  auto bail = [&](int code) {
    if (c->h_ctl) (void)hipHostFree(c->h_ctl);
    if (c->h_ring) (void)hipHostFree(c->h_ring);
    delete c;
    return code;
  };
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_ctl), sizeof(Control), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c->h_ring), RING_CAP * 8 * sizeof(double), hipHostMallocDefault) !=
          hipSuccess)
    return bail(RELAX_E_HIP);

  const size_t N3 = 3 * (size_t)c->g.N;
  if (hipMemcpyAsync(c->d_x[0], d_x0, N3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->d_B0_64, d_B0, N3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return bail(RELAX_E_HIP);
  // max |B0|^2 of the caller's field (null guard of xi), then B0 -> B0'' = B0 * 4 h_b h_c for
  // the unscaled-difference form of the sweep
  if (launch_max_norm2(c->d_B0_64, c->g.N, c->d_out, c->d_part, c->g.nblocks * NPART, c->stream) != hipSuccess)
    return bail(RELAX_E_HIP);
  if (launch_prescale(c->d_B0_64, c->g.N, c->g.b0scale, c->stream) != hipSuccess) return bail(RELAX_E_HIP);
  if (c->mixed && launch_to_float(c->d_B0_64, static_cast<float*>(c->d_B0), (long long)N3, c->stream) != hipSuccess)
    return bail(RELAX_E_HIP);
  if (hipMemcpyAsync(c->h_ring, c->d_out, sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return bail(RELAX_E_HIP);
  const double maxB2 = c->h_ring[0];
  if (!std::isfinite(maxB2)) return bail(RELAX_E_NAN);

  Control& k = *c->h_ctl;
  std::memset(&k, 0, sizeof(Control));
  k.t = 0.0;
  k.dt = cfg->dt0;
  k.tol = cfg->tol;
  k.safety = cfg->safety;
  k.dt_min = cfg->dt_min;
  k.gamma = cfg->gamma;
  k.tau_B2 = cfg->xi_null_tau * maxB2;
  k.dV = c->g.dV;
  k.status = 0;
  k.cur = 0;
  k.need_k1 = 1;
  k.adaptive = cfg->adaptive;
  k.record = (L.ckpt_slots > 0) ? 1 : 0;
  k.ck_every = std::max(1, cfg->checkpoint_every);
  k.record_cap = c->K_record;
  k.steps_total = 0;
  if ((rc = push_ctl(c)) != RELAX_OK) return bail(rc);
  double d[6];
  if ((rc = diagnostics_sweep(c, 0, d)) != RELAX_OK) return bail(rc);
  if (d[3] != d[3] || !std::isfinite(d[0])) return bail(RELAX_E_NAN);
  if (!(d[3] > 0.0)) return bail(RELAX_E_FOLD);
  *out_ctx = c;
  return RELAX_OK;
}

int relax_step(void* ctx, int K, relax_diag* host_diag, int* steps_done) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (steps_done) *steps_done = 0;
  if (!c || K < 0) return RELAX_E_ARG;
  if (c->status != RELAX_OK) return RELAX_E_STATE;
  int done = 0, rc = RELAX_OK;
  while (done < K) {
    const int chunk = std::min(K - done, RING_CAP);
    HIP_TRY(c, launch_begin_chunk(c->d_ctl, chunk, c->stream));
    int pending = chunk;
    for (;;) {
      if ((rc = enqueue_attempts(c, pending)) != RELAX_OK) return rc;
      if ((rc = sync_ctl(c)) != RELAX_OK) return rc;
      if (c->profiling && (rc = prof_harvest(c)) != RELAX_OK) return rc;
      if (c->h_ctl->status != 0 || c->h_ctl->accepted >= chunk) break;
      pending = chunk - c->h_ctl->accepted;
    }
    const int acc = c->h_ctl->accepted;
    if (host_diag && acc > 0) {
      HIP_TRY(c, hipMemcpyAsync(c->h_ring, c->d_ring, (size_t)acc * 8 * sizeof(double), hipMemcpyDeviceToHost,
                                c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      for (int i = 0; i < acc; i++) {
        const double* e = c->h_ring + 8 * i;
        relax_diag& o = host_diag[done + i];
        o.t = e[0];
        o.dt = e[1];
        o.E_M = e[2];
        o.xi = e[3];
        o.R2 = e[4];
        o.Lambda = e[5];
        o.min_det = e[6];
        o.rejects = (int)e[7];
        o.concave = 0;
      }
    }
    done += acc;
    if (steps_done) *steps_done = done;
    if (c->h_ctl->status != 0) {
      const int code = c->h_ctl->status;
      const char* what = code == RELAX_E_FOLD ? "folded grid (min det F <= 0)"
                         : code == RELAX_E_DT ? "step size fell below dt_min"
                                              : "non-finite energy, residual or error estimate";
      return fail(c, code, std::string("relax_step: ") + what + " after " + std::to_string(done) + " steps");
    }
  }
  return RELAX_OK;
}

int relax_diagnostics(void* ctx, relax_diag* out) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || !out) return RELAX_E_ARG;
  if (c->status != RELAX_OK) return RELAX_E_STATE;
  int rc = sync_ctl(c);
  if (rc) return rc;
  double d[6];
  if ((rc = diagnostics_sweep(c, c->cur, d)) != RELAX_OK) return rc;
  out->t = c->h_ctl->t;
  out->dt = c->h_ctl->dt;
  out->E_M = d[0];
  out->R2 = d[1];
  out->xi = d[2];
  out->min_det = d[3];
  out->Lambda = 0.0;
  out->rejects = 0;
  out->concave = (int)d[5];
  return RELAX_OK;
}

int relax_velocity(void* ctx, double* d_u_out) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || !d_u_out) return RELAX_E_ARG;
  if (c->status != RELAX_OK) return RELAX_E_STATE;
  int rc = sync_ctl(c);
  if (rc) return rc;
  double d[6];
  return diagnostics_sweep(c, c->cur, d, d_u_out);
}

int relax_fields(void* ctx, double* d_B_out, double* d_J_out) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return RELAX_E_ARG;
  if (c->status != RELAX_OK) return RELAX_E_STATE;
  int rc = sync_ctl(c);
  if (rc) return rc;
  double d[6];
  return diagnostics_sweep(c, c->cur, d, nullptr, 0.0, d_B_out, d_J_out);
}

int relax_monitors(void* ctx, double* d_alpha_out, int* d_kappa_out) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return RELAX_E_ARG;
  if (c->status != RELAX_OK) return RELAX_E_STATE;
  int rc = sync_ctl(c);
  if (rc) return rc;
  double d[6];
  return diagnostics_sweep(c, c->cur, d, nullptr, 0.0, nullptr, nullptr, d_alpha_out, d_kappa_out);
}

int relax_backward(void* ctx, double seed_EM, double seed_R2, double* d_grad_x0, double* d_grad_B0) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || !d_grad_x0 || !d_grad_B0 || !std::isfinite(seed_EM) || !std::isfinite(seed_R2)) return RELAX_E_ARG;
  if (c->status != RELAX_OK) return RELAX_E_STATE;
  if (c->mixed) return fail(c, RELAX_E_ARG, "relax_backward: needs an FP64 context");
  if (c->cfg.curl != RELAX_CURL_NN) return fail(c, RELAX_E_ARG, "relax_backward: nearest-neighbour current only");
  if (c->L.ckpt_slots == 0) return fail(c, RELAX_E_STATE, "relax_backward: context created without record");
  if (seed_R2 != 0.0 && c->cfg.gamma == 0.0) return fail(c, RELAX_E_ARG, "relax_backward: R2 seed needs gamma != 0");
  int rc = sync_ctl(c);
  if (rc) return rc;
  const long long K = c->h_ctl->steps_total;
  if (K > c->K_record) return fail(c, RELAX_E_STATE, "relax_backward: more steps taken than K_record");
  const long long N = c->g.N;
  const size_t N3 = 3 * (size_t)N;
  const int cpe = c->cfg.checkpoint_every;
  hipStream_t st = c->stream;

  AdjArgs a{};
  a.g = c->g;
  a.B0 = c->d_B0_64;
  a.Fbar = c->d_Fbar;
  a.B0bar = c->d_B0bar;
  a.gamma = c->cfg.gamma;
  a.seed_EM = seed_EM;
  a.seed_R2 = seed_R2;
  a.xbar = c->d_xbar;
  for (int t = 2; t <= 6; t++) a.ybar[t] = c->d_ybar + (size_t)(t - 2) * N3;
  a.ubar = c->d_ubar;
  a.ubar_out = c->d_ubar;
  HIP_TRY(c, launch_fill(c->d_B0bar, (long long)N3, 0.0, st));

  // seed: cotangents of E_M(x_K) and R2(x_K)
  a.useed = nullptr;
  if (seed_R2 != 0.0) {
    double d[6];
    const double gm = c->cfg.gamma;
    if ((rc = diagnostics_sweep(c, c->cur, d, c->d_useed, c->g.dV * seed_R2 / (gm * gm))) != RELAX_OK) return rc;
    a.useed = c->d_useed;
  }
  a.x = c->d_x[c->cur];
  HIP_TRY(c, launch_adj_field(1, true, a, st));
  a.xbar_out = c->d_xbar;
  HIP_TRY(c, launch_adj_gather(a, 2, 1, st));
  a.useed = nullptr;

  // reverse over the recorded steps, one checkpoint segment at a time
  HIP_TRY(c, hipMemcpyAsync(c->d_ctl2, c->d_ctl, sizeof(Control), hipMemcpyDeviceToDevice, st));
  SweepArgs fw = sweep_args(c);
  fw.ctl = c->d_ctl2;
  fw.B0 = c->d_B0_64;
  fw.ckpt = nullptr;
  fw.ckpt_slots = 0;
  const long long nseg = (K + cpe - 1) / cpe;
  for (long long seg = nseg - 1; seg >= 0; seg--) {
    const long long s0 = seg * cpe, s1 = std::min<long long>(s0 + cpe, K);
    const int len = (int)(s1 - s0);
    HIP_TRY(c, hipMemcpyAsync(c->d_seg_x, c->d_ckpt + (size_t)seg * N3, N3 * sizeof(double),
                              hipMemcpyDeviceToDevice, st));
    // forward recompute, keeping x_n, k_1..k_3 and y_3..y_6 of every step
    for (int j = 0; j < len; j++) {
      HIP_TRY(c, launch_seg_step(c->d_ctl2, c->d_dtrec, s0 + j, st));
      fw.x[0] = c->d_seg_x + (size_t)j * N3;
      fw.x[1] = c->d_seg_x + (size_t)(j + 1) * N3;
      fw.xout[0] = c->d_seg_x + (size_t)j * N3;
      fw.xout[1] = c->d_seg_x + (size_t)(j + 1) * N3;
      for (int s = 0; s < 3; s++) fw.k[s] = c->d_seg_k + ((size_t)j * 3 + s) * N3;
      // y_3 .. y_6 of step j: stages 2 and 4 write y_3 and y_5 there; stages 4 and 6 add y_4, y_6
      double* ys = c->d_seg_y + (size_t)j * 4 * N3;
      fw.y3 = ys;
      fw.yrec[0] = ys + N3;
      fw.y5 = ys + 2 * N3;
      fw.yrec[1] = ys + 3 * N3;
      for (int s = 1; s <= 6; s++) HIP_TRY(c, launch_stage_rec(s, fw, st));
    }
    for (int j = len - 1; j >= 0; j--) {
      a.x = c->d_seg_x + (size_t)j * N3;
      for (int s = 0; s < 3; s++) a.k[s] = c->d_seg_k + ((size_t)j * 3 + s) * N3;
      for (int t = 0; t < 4; t++) a.y[t] = c->d_seg_y + ((size_t)j * 4 + t) * N3;
      a.dt = c->d_dtrec + s0 + j;
      for (int s = 6; s >= 1; s--) {
        HIP_TRY(c, launch_adj_field(s, false, a, st));
        if (s >= 2) {
          a.ybar_out = c->d_ybar + (size_t)(s - 2) * N3;
          HIP_TRY(c, launch_adj_gather(a, 0, s, st));
        } else {
          a.xbar_out = c->d_xbar;
          HIP_TRY(c, launch_adj_gather(a, 1, 1, st));
        }
      }
    }
  }
  HIP_TRY(c, hipMemcpyAsync(d_grad_x0, c->d_xbar, N3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIP_TRY(c, hipMemcpyAsync(d_grad_B0, c->d_B0bar, N3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIP_TRY(c, launch_prescale(d_grad_B0, N, c->g.b0scale, st));  // d/dB0 = 4 h_b h_c d/dB0''
  HIP_TRY(c, hipStreamSynchronize(st));
  return RELAX_OK;
}

int relax_get_state(void* ctx, double* d_x_out, double* t, double* dt) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return RELAX_E_ARG;
  int rc = sync_ctl(c);
  if (rc) return rc;
  if (d_x_out) {
    HIP_TRY(c, hipMemcpyAsync(d_x_out, c->d_x[c->cur], 3 * (size_t)c->g.N * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  if (t) *t = c->h_ctl->t;
  if (dt) *dt = c->h_ctl->dt;
  return RELAX_OK;
}

int relax_set_state(void* ctx, const double* d_x_in, double t, double dt) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || !d_x_in || !std::isfinite(t) || !(dt > 0.0) || !std::isfinite(dt)) return RELAX_E_ARG;
  int rc = sync_ctl(c);
  if (rc && c->h_ctl == nullptr) return rc;
  c->status = RELAX_OK;
  c->err.clear();
  HIP_TRY(c, hipMemcpyAsync(c->d_x[0], d_x_in, 3 * (size_t)c->g.N * sizeof(double), hipMemcpyDeviceToDevice,
                            c->stream));
  Control& k = *c->h_ctl;
  k.t = t;
  k.dt = dt;
  k.status = 0;
  k.cur = 0;
  k.need_k1 = 1;
  k.rejects = 0;
  k.accepted = 0;
  k.target = 0;
  k.steps_total = 0;
  if ((rc = push_ctl(c)) != RELAX_OK) return rc;
  c->cur = 0;
  double d[6];
  if ((rc = diagnostics_sweep(c, 0, d)) != RELAX_OK) return rc;
  if (d[3] != d[3] || !std::isfinite(d[0])) return fail(c, RELAX_E_NAN, "relax_set_state: non-finite state");
  if (!(d[3] > 0.0)) return fail(c, RELAX_E_FOLD, "relax_set_state: folded grid (min det F <= 0)");
  return RELAX_OK;
}

int relax_profile(void* ctx, int on, double* ms_out, long long* launches_out) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c || (on != 0 && on != 1)) return RELAX_E_ARG;
  for (int k = 0; k < 7; k++) {
    if (ms_out) ms_out[k] = c->prof_ms[k];
    if (launches_out) launches_out[k] = c->prof_n[k];
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  c->profiling = (on != 0);
  return RELAX_OK;
}

const char* relax_strerror(int code) {
  switch (code) {
    case RELAX_OK: return "ok";
    case RELAX_E_ARG: return "invalid argument";
    case RELAX_E_HIP: return "HIP runtime error";
    case RELAX_E_FOLD: return "folded grid: min det F <= 0";
    case RELAX_E_DT: return "step size below dt_min";
    case RELAX_E_NAN: return "non-finite energy, residual or error estimate";
    case RELAX_E_STATE: return "context failed or nothing recorded";
    case RELAX_E_SPACE: return "workspace too small";
    default: return "unknown status";
  }
}

const char* relax_last_error(void* ctx) {
  Ctx* c = static_cast<Ctx*>(ctx);
  return c ? c->err.c_str() : "";
}

void relax_destroy(void* ctx) {
  Ctx* c = static_cast<Ctx*>(ctx);
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->h_ctl) (void)hipHostFree(c->h_ctl);
  if (c->h_ring) (void)hipHostFree(c->h_ring);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"
