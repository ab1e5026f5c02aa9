// stage.hip -- the fused Runge-Kutta stage sweep of the mimetic magneto-frictional step.
//
// One launch evaluates, for every node, the right-hand side u = gamma J x B of the
// Lagrangian relaxation (eq. "magneto friction") at the stage input
//     y_s = x_n + dt sum_{j<s} a_sj k_j                  (Cash-Karp RK5(4), Sec. 2.4)
// and stores what the later stages need.  Stage 1 also reduces the diagnostics of x_n (E_M
// with the face weights zeta, eq. "magnetic energy"; xi = max |J x B| / B^2; R2; min Delta);
// stage 6 writes x_{n+1} with the fifth-order weights and reduces the embedded error
// Lambda = max |x5 - x4|.
//
// Per node the operator is two radius-1 stencils joined by pointwise maps.  With the
// UNSCALED differences (the 1/(2h) factors cancel):
//   F'   = differences of y: y(n+e_a) - y(n-e_a), or the one-sided second-order rows
//          -3y0 + 4y1 - y2 / 3y0 - 4y1 + y2 on line-tied end nodes; on periodic axes the
//          neighbour carries the +-period coordinate shift (Sec. 2.5).  F' = F diag(2h).
//   B    = F' B0'' / det F'  with B0''_a = 4 h_b h_c B0_a, which equals F B0 / det F
//          (eq. "B transformation")
//   G'_a = B(n+e_a) - B(n-e_a)
//   J    = F' c' / det F',   c'_q = (F' e_b) . G'_a - (F' e_a) . G'_b,  (a, b, q) cyclic.
// The last line is the Stokes-loop current of Sec. 2.2 (eqs. "current discrete", "four
// surfaces", "current matrix equation") in closed form: on the diamond of the four
// in-plane neighbours the edge-averaged circulation is 2 h_a h_b c_q and the sum of the
// four triangle vectors is 2 h_a h_b (F e_a) x (F e_b) = 2 h_a h_b cof(F) e_q, so the
// paper's 3x3 system is (cof F)^T J = c, solved by J = F c / det F; with F = F' diag(1/2h)
// and G = G' diag(1/2h) every spacing factor cancels.
//
// Stage inputs.  Every stage input is x_n plus ONE rounded increment, y_s = x_n + d_s with
// d_s = dt sum_j a_sj k_j summed first: the stencil differentiates y_s twice, and on a fine
// grid a rounding of y_s is amplified by about 1/h^2 in u, so the inputs are rounded once from
// x_n (as the plain definition does) and never accumulated stage by stage.  A stencilled
// window holds at most two vectors (more overflow each XCD's L2 with halo lines); what a
// stage needs at its output node from its own window (x_n, and k_1 in stage 2) is carried in
// registers from the window load, three plane steps earlier, instead of being read again.
//   stage 1: window x_n                    -> k_1
//   stage 2: window x_n + dt a_21 k_1      -> k_2, y_3 = x_n + dt (a_31 k_1 + a_32 k_2)
//   stage 3: window y_3; k_1, k_2 at node  -> k_3, d_4 = dt (a_41 k_1 + a_42 k_2 + a_43 k_3)
//   stage 4: window x_n + d_4; k_1..k_3    -> y_5 = x_n + d_5 and the partial sums of k_1..k_4
//            P6 = dt sum a_6j k_j, X = dt sum b5_j k_j, E = dt sum (b5_j - b4_j) k_j
//   stage 5: window y_5; P6, E at node     -> P6 += dt a_65 k_5 (now d_6), E += dt (b5_5 - b4_5) k_5
//   stage 6: window x_n + d_6; X, E        -> x_{n+1} = x_n + (X + dt b5_6 k_6),
//                                             Lambda = max |E + dt (b5_6 - b4_6) k_6|
// k_4, k_5 and k_6 are never stored.  HBM bytes per node and attempt: 864 (FP64), 540
// (FP32-mixed: the k_j, d_4 and the partial sums in FP32; x_n, y_3 and y_5 in FP64).  x_{n+1}
// is x_n plus an increment built from the k_j alone, so the step keeps full relative precision
// however small it is.  A retried step (smaller dt, same x_n and k_1) starts again at stage 2,
// and every stored vector is rewritten before it is read again.  REC (the forward replay of
// the reverse pass) also stores y_4 and y_6 at the node for the reverse sweeps.
//
// Data flow: a workgroup owns a 64 x 8 (x, y) tile and marches up a z-chunk.  Each plane
// of the stage input (tile + 2-node halo, FP64) goes into an LDS ring of three planes;
// F', det F' and B are formed on the tile + 1-node halo into an LDS ring of two B planes
// (the z difference of B at the tile node uses the node's own B of the neighbouring
// planes, kept in registers); the current, force and velocity are formed on the tile one
// plane behind.  Every global access is a buffer instruction whose masked-off lanes carry
// an offset past the record count (loads return 0, stores are dropped), so the march has
// no divergent branch around a memory instruction: each load is issued one plane step
// before its use, in the same order on every step, and waited for by exact counts.
#include <type_traits>

#include "sweep_common.h"

namespace relax {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) {
    double w = __shfl_xor(v, o, 64);
    v = (w > v || w != w) ? w : v;
  }
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) {
    double w = __shfl_xor(v, o, 64);
    v = (w < v || w != w) ? w : v;
  }
  return v;
}

// S: stage 1..6.  MIXED: the k_j, the partial sums and B0 in FP32, and the stencil past F' in
// FP32.  XYP: x and y both periodic (no line-tied rows in x and y).  DIAG (stage 1, FP64): the
// diagnostics sweep of x[diag_buf]: no step gating and no k_1; writes u (optionally scaled by
// det F), B, J, alpha* and the convexity where the caller asked for them.  REC (FP64 stages
// 4 and 6): also store the stage input at the node, for the reverse sweeps.
template <int S, bool MIXED, bool XYP, bool DIAG = false, bool REC = false, bool NNN = false>
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(2))) void stage_kernel(SweepArgs a) {
  using T = typename std::conditional<MIXED, float, double>::type;
  // NNN: the current from the next-nearest-neighbour octilateral loops (Sec. 2.3), which reach
  // positions and B on the planes q - 1 and q + 1 with an x-y offset: the stage-input ring
  // keeps five planes and the B ring three
  constexpr int RYS = NNN ? 5 : 3;
  constexpr int RBS = NNN ? 3 : 2;
  auto yslot = [](int p) { return (int)((unsigned)(p + 1024 * RYS) % (unsigned)RYS); };
  auto bslot = [](int p) { return (int)((unsigned)(p + 1024 * RBS) % (unsigned)RBS); };
  constexpr bool STAGE1 = (S == 1);
  constexpr bool LAST = (S == 6);
  // the window is a base vector (x_n; y_3 in stage 3, y_5 in stage 5) plus at most one vector
  // v with coefficient cv: k_1 (cv = dt a_21) in stage 2, d_4 and d_6 (cv = 1) in stages 4, 6
  constexpr bool WV = (S == 2 || S == 4 || LAST);
  // own-node values carried from the window to the output node (3 planes later): x_n in
  // stages 2, 4, 6 (and k_1 in stage 2)
  constexpr bool CX = WV;
  constexpr bool CK1 = (S == 2);
  constexpr int NPK = (S == 3) ? 2 : (S == 4 ? 3 : 0);  // k_j read at the output node
  constexpr int NPKA = NPK > 0 ? NPK : 1;
  constexpr bool PS = (S == 5 || LAST);  // two partial sums read at the output node
  constexpr bool SUMS_OUT = (S == 3 || S == 4 || S == 5);
  constexpr int NP2 = (RY2 * RX2 + NTHREADS - 1) / NTHREADS;  // stage-input points per thread
  constexpr int NP1 = (RY1 * RX1 + NTHREADS - 1) / NTHREADS;  // field points per thread
  static_assert(!DIAG || (S == 1 && !MIXED), "the diagnostics sweep is the FP64 stage-1 sweep");
  static_assert(!REC || (!MIXED && (S == 4 || S == 6)), "REC: FP64 stages 4 and 6");
  static_assert(!NNN || (!MIXED && !REC), "the octilateral current is an FP64 forward operator");

  Control* ctl = a.ctl;
  constexpr bool diag_only = DIAG;
  int cur;
  double dt = 0.0;
  bool record_ck = false;
  long long ck_slot = 0;
  if (!diag_only) {
    if (ctl->status != 0 || ctl->accepted >= ctl->target) return;
    if (STAGE1 && ctl->need_k1 == 0) return;
    cur = ctl->cur;
    dt = ctl->dt;
    if (STAGE1 && ctl->record) {
      const long long st = ctl->steps_total;
      if (st % ctl->ck_every == 0 && st / ctl->ck_every < a.ckpt_slots) {
        record_ck = true;
        ck_slot = st / ctl->ck_every;
      }
    }
  } else {
    cur = a.diag_buf;
  }
  const double gamma = ctl->gamma;
  const double tau_B2 = ctl->tau_B2;
  const double cv = (S == 2) ? dt * CK::a[1][0] : 1.0;

  const Geometry& g = a.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const long long N = g.N;
  const int bcx = XYP ? BC_PERIODIC : g.bc[0];
  const int bcy = XYP ? BC_PERIODIC : g.bc[1];
  const int bcz = g.bc[2];
  const double inv8h3 = g.inv8h3;
  const unsigned nxy = (unsigned)nx * (unsigned)ny;

  const int lb = logical_block(blockIdx.x, g.nblocks);
  const int tile_x = lb % g.tiles[0];
  const int tile_y = (lb / g.tiles[0]) % g.tiles[1];
  const int chunk = lb / (g.tiles[0] * g.tiles[1]);
  const int i0 = tile_x * TX, j0 = tile_y * TY;
  const int z0 = chunk * g.tz;
  const int z1 = min(z0 + g.tz, nz);

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;

  __shared__ double ys[RYS][3][RY2 * RX2];  // stage input, tile + 2-node halo, ring of planes
  __shared__ T bs[RBS][3][RY1 * RX1];       // pulled-back field, tile + 1-node halo, ring of planes
  __shared__ double red[NTHREADS / 64][NPART];

  const double* __restrict__ xn = a.x[cur];
  const double* __restrict__ wbase = (S == 3) ? a.y3 : ((S == 5) ? a.y5 : xn);  // the window base
  const T* __restrict__ wvec = static_cast<const T*>(S == 2 ? a.k[0] : (S == 4 ? a.d4 : a.sum[0]));
  const T* __restrict__ b0p = static_cast<const T*>(a.B0);

  // plane index of a load (line-tied z: clamped; such planes are loaded but never used)
  auto zload = [&](int pz) {
    if (bcz == BC_PERIODIC) return resolve_near(pz, nz, bcz).i;
    return min(max(pz, 0), nz - 1);
  };

  // ---- per-thread index tables: the (x, y) part of every address is the same on all planes.
  // Window point e, row-major over the window; in the stages that carry own-node values,
  // e < NTHREADS is the tile node of thread e instead (each thread loads its own node), then
  // the two rows below and the two above the tile, then the two columns on either side.
  unsigned w2e[NP2];  // stage-input window point -> flat (x, y) index, IE off the grid
  int w2w[NP2];       // its periodic wraps: x in the low 16 bits, y in the high 16 bits (signed)
  int w2o[NP2];       // its LDS offset, -1 past the window
#pragma unroll
  for (int r = 0; r < NP2; r++) {
    const int e = tid + r * NTHREADS;
    int row, col;
    if (!CX) {
      row = e / RX2;
      col = e - row * RX2;
    } else if (e < NTHREADS) {
      row = e / TX + 2;
      col = e % TX + 2;
    } else {
      const int e2 = e - NTHREADS;
      if (e2 < 4 * RX2) {
        const int band = e2 / RX2;
        row = band < 2 ? band : RY2 - 4 + band;
        col = e2 - band * RX2;
      } else {
        const int e3 = e2 - 4 * RX2, side = e3 & 3;
        row = 2 + (e3 >> 2);
        col = side < 2 ? side : RX2 - 4 + side;
      }
    }
    const bool in_win = e < RY2 * RX2;
    const AxisIdx rx = resolve(i0 + col - 2, nx, bcx);
    const AxisIdx ry = resolve(j0 + row - 2, ny, bcy);
    w2e[r] = (in_win && rx.ok && ry.ok) ? (unsigned)(ry.i * nx + rx.i) : IE;
    w2w[r] = (ry.w << 16) + (rx.w & 0xffff);
    w2o[r] = in_win ? row * RX2 + col : -1;
  }
  // field point e: e < NTHREADS is the tile node of thread e; the rest is the halo ring
  unsigned f1e[NP1];
  int f1r[NP1], f1c[NP1];
#pragma unroll
  for (int r = 0; r < NP1; r++) {
    const int e = tid + r * NTHREADS;
    int r1, c1;
    if (e < NTHREADS) {
      r1 = e / TX + 1;
      c1 = e % TX + 1;
    } else {
      const int e2 = e - NTHREADS;
      if (e2 < RX1) {
        r1 = 0;
        c1 = e2;
      } else if (e2 < 2 * RX1) {
        r1 = RY1 - 1;
        c1 = e2 - RX1;
      } else {
        const int e3 = e2 - 2 * RX1;
        r1 = 1 + (e3 >> 1);
        c1 = (e3 & 1) ? RX1 - 1 : 0;
      }
    }
    const AxisIdx rx = resolve(i0 + c1 - 1, nx, bcx), ry = resolve(j0 + r1 - 1, ny, bcy);
    f1e[r] = (e < RY1 * RX1 && rx.ok && ry.ok) ? (unsigned)(ry.i * nx + rx.i) : IE;
    f1r[r] = (e < RY1 * RX1) ? r1 : -1;
    f1c[r] = c1;
  }

  // tile node owned by this thread
  const int gi_t = i0 + tx, gj_t = j0 + ty;
  const bool tile_ok = (gi_t < nx) && (gj_t < ny);
  const unsigned out_e = tile_ok ? (unsigned)(gj_t * nx + gi_t) : IE;
  const bool face_xy = !XYP && ((bcx == BC_LINE_TIED && (gi_t == 0 || gi_t == nx - 1)) ||
                                (bcy == BC_LINE_TIED && (gj_t == 0 || gj_t == ny - 1)));

  // ---- loads of one plane, issued one plane step ahead of their use -------------------------
  double wx[NP2][3];      // window base (x_n, y_3 or y_5)
  T wk[WV ? NP2 : 1][3];  // the window vector v
  T b0r[NP1][3];          // B0'' at the field points
  T pk[NPKA][3];          // k_j at the output node (stages 3, 4)
  T ps[PS ? 2 : 1][3];    // stage 5: (P6, E); stage 6: (X, E) at the output node
  // own-node values of the three committed planes hi - 2, hi - 1, hi (oldest first)
  double cx[CX ? 3 : 1][3] = {};
  T ck[CK1 ? 3 : 1][3] = {};
  auto load_window = [&](int pz) {
    const long long zo = (long long)zload(pz) * nxy;
#pragma unroll
    for (int m = 0; m < 3; m++) {
      const auto rs = plane_rsrc(wbase + m * N + zo, nxy);
#pragma unroll
      for (int r = 0; r < NP2; r++) wx[r][m] = bload<double>(rs, w2e[r]);
    }
    if constexpr (WV) {
#pragma unroll
      for (int m = 0; m < 3; m++) {
        const auto rs = plane_rsrc(wvec + m * N + zo, nxy);
#pragma unroll
        for (int r = 0; r < NP2; r++) wk[r][m] = bload<T>(rs, w2e[r]);
      }
    }
  };
  // y = base + cv v, rounded once, plus the periodic shift of a wrapped neighbour
  auto commit_window = [&](int pz) {
    const AxisIdx rz = resolve_near(pz, nz, bcz);
    const int slot = yslot(pz);
    const double shz = rz.w * g.period[2];
#pragma unroll
    for (int r = 0; r < NP2; r++) {
      const bool ok = (w2e[r] != IE);
      double v[3];
#pragma unroll
      for (int m = 0; m < 3; m++) {
        double y = wx[r][m];
        if constexpr (S == 2) {
          y = y + cv * (double)wk[r][m];
        } else if constexpr (WV) {
          y = y + (double)wk[r][m];
        }
        v[m] = y;
      }
      v[0] += (double)(short)(w2w[r] & 0xffff) * g.period[0];
      v[1] += (double)(w2w[r] >> 16) * g.period[1];
      v[2] += shz;
      if (w2o[r] >= 0) {
#pragma unroll
        for (int m = 0; m < 3; m++) ys[slot][m][w2o[r]] = ok ? v[m] : 0.0;
      }
    }
    // the own node (window point 0) enters the carry
#pragma unroll
    for (int m = 0; m < 3; m++) {
      if constexpr (CX) {
        cx[0][m] = cx[1][m];
        cx[1][m] = cx[2][m];
        cx[2][m] = wx[0][m];
      }
      if constexpr (CK1) {
        ck[0][m] = ck[1][m];
        ck[1][m] = ck[2][m];
        ck[2][m] = wk[0][m];
      }
    }
  };
  auto load_b0 = [&](int pz) {
    const long long zo = (long long)zload(pz) * nxy;
#pragma unroll
    for (int m = 0; m < 3; m++) {
      const auto rs = plane_rsrc(b0p + m * N + zo, nxy);
#pragma unroll
      for (int r = 0; r < NP1; r++) b0r[r][m] = bload<T>(rs, f1e[r]);
    }
  };
  auto load_point = [&](int pz) {
    const long long zo = (long long)zload(pz) * nxy;
    if constexpr (NPK > 0) {
#pragma unroll
      for (int j = 0; j < NPK; j++) {
        const T* kj = static_cast<const T*>(a.k[j]);
#pragma unroll
        for (int m = 0; m < 3; m++) pk[j][m] = bload<T, CPOL_STREAM>(plane_rsrc(kj + m * N + zo, nxy), out_e);
      }
    }
    if constexpr (PS) {
      const T* s0 = static_cast<const T*>(S == 5 ? a.sum[0] : a.sum[1]);
      const T* s1 = static_cast<const T*>(a.sum[2]);
#pragma unroll
      for (int m = 0; m < 3; m++) ps[0][m] = bload<T, CPOL_STREAM>(plane_rsrc(s0 + m * N + zo, nxy), out_e);
#pragma unroll
      for (int m = 0; m < 3; m++) ps[1][m] = bload<T, CPOL_STREAM>(plane_rsrc(s1 + m * N + zo, nxy), out_e);
    }
  };

  // ---- unscaled Jacobian at a window point (r, c in stage-input window coordinates) -----
  auto jac_xy = [&](int r, int c, int p, int gi, int gj, double F[3][3]) {
    const int o = r * RX2 + c;
    const int sp = yslot(p);
#pragma unroll
    for (int m = 0; m < 3; m++) {
      const double* yc = ys[sp][m];
      if (XYP || bcx == BC_PERIODIC || (gi > 0 && gi < nx - 1))
        F[m][0] = yc[o + 1] - yc[o - 1];
      else if (gi == 0)
        F[m][0] = -3.0 * yc[o] + 4.0 * yc[o + 1] - yc[o + 2];
      else
        F[m][0] = 3.0 * yc[o] - 4.0 * yc[o - 1] + yc[o - 2];
      if (XYP || bcy == BC_PERIODIC || (gj > 0 && gj < ny - 1))
        F[m][1] = yc[o + RX2] - yc[o - RX2];
      else if (gj == 0)
        F[m][1] = -3.0 * yc[o] + 4.0 * yc[o + RX2] - yc[o + 2 * RX2];
      else
        F[m][1] = 3.0 * yc[o] - 4.0 * yc[o - RX2] + yc[o - 2 * RX2];
    }
  };
  auto jacobian = [&](int r, int c, int p, int gi, int gj, double F[3][3]) {
    jac_xy(r, c, p, gi, gj, F);
    const int o = r * RX2 + c;
    if (bcz == BC_PERIODIC || (p > 0 && p < nz - 1)) {
      const int sa = yslot(p + 1), sb = yslot(p - 1);
#pragma unroll
      for (int m = 0; m < 3; m++) F[m][2] = ys[sa][m][o] - ys[sb][m][o];
    } else if (p == 0) {
#pragma unroll
      for (int m = 0; m < 3; m++) F[m][2] = -3.0 * ys[yslot(0)][m][o] + 4.0 * ys[yslot(1)][m][o] - ys[yslot(2)][m][o];
    } else {
      const int s0 = yslot(p), s1 = yslot(p - 1), s2 = yslot(p - 2);
#pragma unroll
      for (int m = 0; m < 3; m++) F[m][2] = 3.0 * ys[s0][m][o] - 4.0 * ys[s1][m][o] + ys[s2][m][o];
    }
  };

  // B planes this chunk needs, and the stage-input window [lo(p), hi(p)] behind each
  const bool perz = (bcz == BC_PERIODIC);
  const int pb0 = perz ? z0 - 1 : max(z0 - 1, 0);
  const int pb1 = perz ? z1 : min(z1, nz - 1);
  auto need_hi = [&](int p) { return perz ? p + 1 : (p == 0 ? 2 : (p == nz - 1 ? p : p + 1)); };
  auto need_lo = [&](int p) { return perz ? p - 1 : (p == 0 ? 0 : (p == nz - 1 ? p - 2 : p - 1)); };

  // reductions
  double acc_E = 0.0, acc_R2 = 0.0, acc_min = INFINITY, acc_null = 0.0, acc_lam = 0.0;
  double acc_conc = 0.0;  // DIAG: concave nodes
  // xi: the node of largest |f|^2 / B^4 so far, kept as (|f|^2, B^4, B^2) and compared by
  // cross-multiplication, so that the square root and the division are taken once at the end
  double xi_F2 = 0.0, xi_B4 = 1.0, xi_B2 = 1.0;
  int kap_q = 1;  // DIAG: convexity of the own node of the output plane q

  // ---- stores of one output plane (every lane issues them; masked-off lanes are dropped) ----
  T so_k[3] = {T(0), T(0), T(0)};    // k_s (stages 1..3), u (DIAG)
  double so_y[3] = {0.0, 0.0, 0.0};  // x_n copy (stage 1), y_3 (stage 2), y_5 (stage 4), x_{n+1}
  T so_s[SUMS_OUT ? 3 : 1][3] = {};  // stage 3: d_4; stage 4: P6, X, E; stage 5: P6, -, E
  double so_p[DIAG ? 3 : 1][3] = {}; // DIAG: B, J, alpha*
  double ycq[3] = {0.0, 0.0, 0.0};   // the stage input at the tile node of plane q
  auto store_plane = [&](int qz, bool on) {
    const long long zo = (long long)zload(qz) * nxy;
    const unsigned eo = on ? out_e : IE;
    if constexpr (DIAG) {
      // each output goes to the caller's array, or (masked) to x[diag_buf], never written
      double* fb = const_cast<double*>(a.x[cur]);
      double* du = a.u_out ? a.u_out : fb;
      double* dB = a.B_out ? a.B_out : fb;
      double* dJ = a.J_out ? a.J_out : fb;
      const unsigned eu = (on && a.u_out) ? out_e : IE, eB = (on && a.B_out) ? out_e : IE;
      const unsigned eJ = (on && a.J_out) ? out_e : IE;
      double* dA = a.alpha_out ? a.alpha_out : fb;
      int* dK = a.kappa_out ? a.kappa_out : reinterpret_cast<int*>(fb);
      const unsigned eA = (on && a.alpha_out) ? out_e : IE, eK = (on && a.kappa_out) ? out_e : IE;
#pragma unroll
      for (int m = 0; m < 3; m++) bstore<double>(plane_rsrc(du + m * N + zo, nxy), eu, (double)so_k[m]);
#pragma unroll
      for (int m = 0; m < 3; m++) bstore<double>(plane_rsrc(dB + m * N + zo, nxy), eB, so_p[0][m]);
#pragma unroll
      for (int m = 0; m < 3; m++) bstore<double>(plane_rsrc(dJ + m * N + zo, nxy), eJ, so_p[1][m]);
      bstore<double>(plane_rsrc(dA + zo, nxy), eA, so_p[2][0]);
      bstore<int>(plane_rsrc(dK + zo, nxy), eK, kap_q);
    } else if constexpr (STAGE1) {
      const unsigned ec = (on && record_ck) ? out_e : IE;
      T* dk = static_cast<T*>(a.k[0]);
      double* dc = record_ck ? a.ckpt + ck_slot * 3 * N : a.xout[0];
#pragma unroll
      for (int m = 0; m < 3; m++) bstore<T>(plane_rsrc(dk + m * N + zo, nxy), eo, so_k[m]);
#pragma unroll
      for (int m = 0; m < 3; m++) bstore<double>(plane_rsrc(dc + m * N + zo, nxy), ec, so_y[m]);
    } else if constexpr (S == 2) {
      T* dk = static_cast<T*>(a.k[1]);
#pragma unroll
      for (int m = 0; m < 3; m++) bstore<T>(plane_rsrc(dk + m * N + zo, nxy), eo, so_k[m]);
#pragma unroll
      for (int m = 0; m < 3; m++) bstore<double>(plane_rsrc(a.y3 + m * N + zo, nxy), eo, so_y[m]);
    } else if constexpr (S == 3) {
      T* dk = static_cast<T*>(a.k[2]);
      T* dd = static_cast<T*>(a.d4);
#pragma unroll
      for (int m = 0; m < 3; m++) bstore<T>(plane_rsrc(dk + m * N + zo, nxy), eo, so_k[m]);
#pragma unroll
      for (int m = 0; m < 3; m++) bstore<T>(plane_rsrc(dd + m * N + zo, nxy), eo, so_s[0][m]);
    } else if constexpr (S == 4) {
#pragma unroll
      for (int m = 0; m < 3; m++) bstore<double>(plane_rsrc(a.y5 + m * N + zo, nxy), eo, so_y[m]);
#pragma unroll
      for (int i = 0; i < 3; i++) {
        T* ds = static_cast<T*>(a.sum[i]);
#pragma unroll
        for (int m = 0; m < 3; m++) bstore<T>(plane_rsrc(ds + m * N + zo, nxy), eo, so_s[i][m]);
      }
    } else if constexpr (S == 5) {
#pragma unroll
      for (int i = 0; i < 3; i += 2) {
        T* ds = static_cast<T*>(a.sum[i]);
#pragma unroll
        for (int m = 0; m < 3; m++) bstore<T>(plane_rsrc(ds + m * N + zo, nxy), eo, so_s[i][m]);
      }
    } else {
      double* xo = a.xout[1 - cur];
#pragma unroll
      for (int m = 0; m < 3; m++) bstore<double>(plane_rsrc(xo + m * N + zo, nxy), eo, so_y[m]);
    }
    if constexpr (REC) {
      double* dy = a.yrec[S == 4 ? 0 : 1];
#pragma unroll
      for (int m = 0; m < 3; m++) bstore<double>(plane_rsrc(dy + m * N + zo, nxy), eo, ycq[m]);
    }
  };

  // ---- prologue: the first stage-input window, synchronously ---------------------------------
  int hi = need_hi(pb0);
  for (int pz = need_lo(pb0); pz <= hi; pz++) {
    load_window(pz);
    commit_window(pz);
  }
  __syncthreads();
  // leave the same loads and (dropped) stores in flight, in the same order, as a plane step
  load_b0(pb0);
  if constexpr (!NNN) load_window(hi + 1);
  load_point(pb0 - 1);
  if constexpr (NNN) load_window(hi + 1);
  store_plane(pb0 - 1, false);

  // own-node values carried between plane steps: B at q - 1 and q; at q: F' z column,
  // 1 / det F', det F
  T Bqm[3] = {T(0), T(0), T(0)}, Bq[3] = {T(0), T(0), T(0)};
  T Fzq[3] = {T(0), T(0), T(0)};
  T rDq = T(0);
  double Dq = 0.0;

  for (int p = pb0; p <= z1; p++) {
    const int q = p - 1;
    const bool qout = (q >= z0 && q < z1);
    // 1. F', det F' and B on the tile + 1-node halo of plane p
    T Bp[3] = {T(0), T(0), T(0)};
    T Fzp[3] = {T(0), T(0), T(0)};
    T rDp = T(0);
    double Dp = 0.0;
    int kap_p = 1;
    if (p <= pb1) {
      const int sb = bslot(p);
#pragma unroll
      for (int r = 0; r < NP1; r++) {
        __builtin_amdgcn_sched_barrier(0);  // one field point at a time: bounds live temporaries
        if (f1r[r] >= 0) {
          const int r1 = f1r[r], c1 = f1c[r];
          const int gi = i0 + c1 - 1, gj = j0 + r1 - 1;
          T B[3] = {T(0), T(0), T(0)};
          if (f1e[r] != IE) {
            double F[3][3];
            jacobian(r1 + 1, c1 + 1, p, gi, gj, F);
            const double D = det3(F);
            const double rD = rcp_nr(D);
            T q0 = b0r[r][0], q1 = b0r[r][1], q2 = b0r[r][2];
            if constexpr (DIAG) {
              q0 *= a.b0_mul[0];
              q1 *= a.b0_mul[1];
              q2 *= a.b0_mul[2];
            }
            if constexpr (MIXED) {
              const float fi = (float)rD;
#pragma unroll
              for (int m = 0; m < 3; m++)
                B[m] = ((float)F[m][0] * q0 + (float)F[m][1] * q1 + (float)F[m][2] * q2) * fi;
            } else {
#pragma unroll
              for (int m = 0; m < 3; m++) B[m] = (F[m][0] * q0 + F[m][1] * q1 + F[m][2] * q2) * rD;
            }
            if (r == 0) {  // this thread's own tile node
#pragma unroll
              for (int m = 0; m < 3; m++) {
                Fzp[m] = (T)F[m][2];
                Bp[m] = B[m];
              }
              rDp = (T)rD;
              Dp = D * inv8h3;
              if (STAGE1 && p >= z0 && p < z1 && gi < nx && gj < ny) {
                // energy in FP64 from the FP64 Jacobian and B0'', weights zeta on line-tied faces
                double zeta = 1.0;
                if (bcx == BC_LINE_TIED && (gi == 0 || gi == nx - 1)) zeta *= 0.5;
                if (bcy == BC_LINE_TIED && (gj == 0 || gj == ny - 1)) zeta *= 0.5;
                if (bcz == BC_LINE_TIED && (p == 0 || p == nz - 1)) zeta *= 0.5;
                double Bd[3];
#pragma unroll
                for (int m = 0; m < 3; m++)
                  Bd[m] = (F[m][0] * (double)q0 + F[m][1] * (double)q1 + F[m][2] * (double)q2) * rD;
                acc_E += zeta * (Bd[0] * Bd[0] + Bd[1] * Bd[1] + Bd[2] * Bd[2]) * Dp;
                acc_min = (Dp < acc_min || Dp != Dp) ? Dp : acc_min;
                if constexpr (DIAG) {
                  // convexity (Sec. 3.2.3, eq. "convexity"): every trihedron of edge vectors to
                  // the neighbours p + di e_x, p + dj e_y, p + dk e_z must have a determinant of
                  // sign di dj dk; trihedra beyond a line-tied face are not formed
                  const int oc = (r1 + 1) * RX2 + (c1 + 1), sc = yslot(p);
                  const bool lox = XYP || bcx == BC_PERIODIC || gi > 0, hix = XYP || bcx == BC_PERIODIC || gi < nx - 1;
                  const bool loy = XYP || bcy == BC_PERIODIC || gj > 0, hiy = XYP || bcy == BC_PERIODIC || gj < ny - 1;
                  const bool loz = bcz == BC_PERIODIC || p > 0, hiz = bcz == BC_PERIODIC || p < nz - 1;
                  double ex[2][3], ey[2][3], ez[2][3];  // [0]: toward -, [1]: toward +
#pragma unroll
                  for (int m = 0; m < 3; m++) {
                    const double c0 = ys[sc][m][oc];
                    ex[0][m] = ys[sc][m][oc - 1] - c0;
                    ex[1][m] = ys[sc][m][oc + 1] - c0;
                    ey[0][m] = ys[sc][m][oc - RX2] - c0;
                    ey[1][m] = ys[sc][m][oc + RX2] - c0;
                    ez[0][m] = loz ? ys[yslot(p - 1)][m][oc] - c0 : 0.0;
                    ez[1][m] = hiz ? ys[yslot(p + 1)][m][oc] - c0 : 0.0;
                  }
                  bool convex = true;
#pragma unroll
                  for (int t = 0; t < 8; t++) {
                    const int a = t & 1, b = (t >> 1) & 1, c = (t >> 2) & 1;
                    const bool formed = (a ? hix : lox) && (b ? hiy : loy) && (c ? hiz : loz);
                    const double* u1 = ex[a];
                    const double* u2 = ey[b];
                    const double* u3 = ez[c];
                    const double det = u1[0] * (u2[1] * u3[2] - u2[2] * u3[1]) - u1[1] * (u2[0] * u3[2] - u2[2] * u3[0]) +
                                       u1[2] * (u2[0] * u3[1] - u2[1] * u3[0]);
                    const double want = ((a + b + c) & 1) ? 1.0 : -1.0;  // (2a-1)(2b-1)(2c-1)
                    if (formed && !(det * want > 0.0)) convex = false;
                  }
                  acc_conc += convex ? 0.0 : 1.0;
                  kap_p = convex ? 1 : -1;
                }
              }
            }
          }
#pragma unroll
          for (int m = 0; m < 3; m++) bs[sb][m][r1 * RX1 + c1] = B[m];
        }
      }
    }
    load_b0(p + 1 <= pb1 ? p + 1 : pb1);
    // x and y columns of F' and the stage input at the tile node of plane q, read before
    // the barrier: the commit below reuses plane q's ring slot
    T Fxy[3][2];
    if (qout) {
      double Ft[3][3];
      jac_xy(ty + 2, tx + 2, q, gi_t, gj_t, Ft);
      const int o = (ty + 2) * RX2 + tx + 2, sq = yslot(q);
#pragma unroll
      for (int m = 0; m < 3; m++) {
        Fxy[m][0] = (T)Ft[m][0];
        Fxy[m][1] = (T)Ft[m][1];
        ycq[m] = ys[sq][m][o];
      }
    }
    __syncthreads();

    // carried own-node values of plane q (the carry holds planes hi - 2, hi - 1, hi), taken
    // before the commit below moves it on
    double xq[3] = {0.0, 0.0, 0.0};
    T kq[3] = {T(0), T(0), T(0)};
    if constexpr (CX) {
      const int cidx = q - (hi - 2);
#pragma unroll
      for (int m = 0; m < 3; m++) {
        xq[m] = cidx == 0 ? cx[0][m] : (cidx == 1 ? cx[1][m] : cx[2][m]);
        if constexpr (CK1) kq[m] = cidx == 0 ? ck[0][m] : (cidx == 1 ? ck[1][m] : ck[2][m]);
      }
    }

    // 2. commit the stage-input plane that field(p + 1) needs; issue the next one
    if (p + 1 <= pb1 && need_hi(p + 1) > hi) {
      hi++;
      commit_window(hi);
    }
    // the octilateral walk below needs many registers: its sweeps load the next window only
    // after it, so that the window buffers are not live across it
    if constexpr (!NNN) load_window(hi + 1);

    // 3. current, force and velocity on the tile of plane q = p - 1
    if (qout) {
      const bool face = face_xy || (bcz == BC_LINE_TIED && (q == 0 || q == nz - 1));
      T u[3] = {T(0), T(0), T(0)};
      if constexpr (DIAG) {
#pragma unroll
        for (int m = 0; m < 3; m++) {
          so_p[0][m] = Bq[m];
          so_p[1][m] = 0.0;  // J: zero on line-tied faces
        }
        so_p[2][0] = 0.0;
      }
      if (!face) {
        const int o = (ty + 1) * RX1 + (tx + 1);
        const int sq = bslot(q);
        T J[3];
        if constexpr (NNN) {
          // the octilateral loops of Sec. 2.3 through the eight ring neighbours of each grid
          // plane, taken literally: vertices V1..V8 = +a, +a+b, +b, -a+b, -a, -a-b, -b, +a-b;
          // circulation sum (B_r + B_r+1)/2 . dx_r; area vector = the triangles at the edge
          // points (V2 V3 V4, V4 V5 V6, V6 V7 V8, V8 V1 V2) plus the quadrilateral through the
          // diagonal points V2 V4 V6 V8; then J . N_q = C_q by Cramer's rule
          const int oy = (ty + 2) * RX2 + tx + 2;
          constexpr int RD[9][2] = {{1, 0}, {1, 1}, {0, 1}, {-1, 1}, {-1, 0}, {-1, -1}, {0, -1}, {1, -1}, {1, 0}};
          double Mq[3][3], Cq[3];
#pragma unroll 1
          for (int qa = 0; qa < 3; qa++) {
            // (a, b) = (y, z), (z, x), (x, y); walk V1..V8 and back to V1, keeping only the
            // previous vertex, the previous edge and the diagonal points met so far
            double Vp[3], Bvp[3], ep[3], e1[3], D1[3], Dp[3], q1[3], qp[3];
            double circ = 0.0, nA[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r <= 8; r++) {
              const int da = RD[r][0], db = RD[r][1];
              const int dx = qa == 2 ? da : (qa == 1 ? db : 0);
              const int dy = qa == 0 ? da : (qa == 2 ? db : 0);
              const int dz = qa == 0 ? db : (qa == 1 ? da : 0);
              const int sy = yslot(q + dz), sbv = bslot(q + dz);
              double V[3], Bv[3];
#pragma unroll
              for (int m = 0; m < 3; m++) {
                V[m] = ys[sy][m][oy + dy * RX2 + dx];
                Bv[m] = (double)bs[sbv][m][o + dy * RX1 + dx];
              }
              if (r > 0) {
                double e[3];
#pragma unroll
                for (int m = 0; m < 3; m++) {
                  e[m] = V[m] - Vp[m];  // dx_r (1-based r), from V_r to V_r+1
                  circ += 0.5 * (Bvp[m] + Bv[m]) * e[m];
                }
                // triangles at the edge points: dx2 x dx3, dx4 x dx5, dx6 x dx7 and dx8 x dx1
                if (r == 3 || r == 5 || r == 7) {
                  nA[0] += 0.5 * (ep[1] * e[2] - ep[2] * e[1]);
                  nA[1] += 0.5 * (ep[2] * e[0] - ep[0] * e[2]);
                  nA[2] += 0.5 * (ep[0] * e[1] - ep[1] * e[0]);
                }
                if (r == 8) {
                  nA[0] += 0.5 * (e[1] * e1[2] - e[2] * e1[1]);
                  nA[1] += 0.5 * (e[2] * e1[0] - e[0] * e1[2]);
                  nA[2] += 0.5 * (e[0] * e1[1] - e[1] * e1[0]);
                }
#pragma unroll
                for (int m = 0; m < 3; m++) {
                  if (r == 1) e1[m] = e[m];
                  ep[m] = e[m];
                }
              }
              // the quadrilateral through the diagonal points V2, V4, V6, V8 (r = 1, 3, 5, 7):
              // edges dx_A..dx_D and the sum of their consecutive cross products over 4
              if (r == 1 || r == 3 || r == 5 || r == 7) {
                if (r == 1) {
#pragma unroll
                  for (int m = 0; m < 3; m++) D1[m] = V[m];
                } else {
                  double qe[3];
#pragma unroll
                  for (int m = 0; m < 3; m++) qe[m] = V[m] - Dp[m];
                  if (r == 3) {
#pragma unroll
                    for (int m = 0; m < 3; m++) q1[m] = qe[m];
                  } else {
                    nA[0] += 0.25 * (qp[1] * qe[2] - qp[2] * qe[1]);
                    nA[1] += 0.25 * (qp[2] * qe[0] - qp[0] * qe[2]);
                    nA[2] += 0.25 * (qp[0] * qe[1] - qp[1] * qe[0]);
                  }
#pragma unroll
                  for (int m = 0; m < 3; m++) qp[m] = qe[m];
                  if (r == 7) {  // the closing edge V8 -> V2, then its products with dx_C and dx_A
                    double qd[3];
#pragma unroll
                    for (int m = 0; m < 3; m++) qd[m] = D1[m] - V[m];
                    nA[0] += 0.25 * (qe[1] * qd[2] - qe[2] * qd[1]) + 0.25 * (qd[1] * q1[2] - qd[2] * q1[1]);
                    nA[1] += 0.25 * (qe[2] * qd[0] - qe[0] * qd[2]) + 0.25 * (qd[2] * q1[0] - qd[0] * q1[2]);
                    nA[2] += 0.25 * (qe[0] * qd[1] - qe[1] * qd[0]) + 0.25 * (qd[0] * q1[1] - qd[1] * q1[0]);
                  }
                }
#pragma unroll
                for (int m = 0; m < 3; m++) Dp[m] = V[m];
              }
#pragma unroll
              for (int m = 0; m < 3; m++) {
                Vp[m] = V[m];
                Bvp[m] = Bv[m];
              }
            }
#pragma unroll
            for (int m = 0; m < 3; m++) Mq[qa][m] = nA[m];
            Cq[qa] = circ;
          }
          const double iM = 1.0 / det3(Mq);
#pragma unroll
          for (int c = 0; c < 3; c++) {
            double Mc[3][3];
#pragma unroll
            for (int r = 0; r < 3; r++)
#pragma unroll
              for (int k = 0; k < 3; k++) Mc[r][k] = (k == c) ? Cq[r] : Mq[r][k];
            J[c] = (T)(det3(Mc) * iM);
          }
        } else {
          T G[3][3];  // G'[a][m] = B_m(n + e_a) - B_m(n - e_a)
#pragma unroll
          for (int m = 0; m < 3; m++) {
            G[0][m] = bs[sq][m][o + 1] - bs[sq][m][o - 1];
            G[1][m] = bs[sq][m][o + RX1] - bs[sq][m][o - RX1];
            G[2][m] = Bp[m] - Bqm[m];
          }
          T Fq[3][3];
#pragma unroll
          for (int m = 0; m < 3; m++) {
            Fq[m][0] = Fxy[m][0];
            Fq[m][1] = Fxy[m][1];
            Fq[m][2] = Fzq[m];
          }
          // c'_q = (F' e_b) . G'_a - (F' e_a) . G'_b, (a, b, q) = (y, z, x), (z, x, y), (x, y, z)
          T cq[3];
          cq[0] = Fq[0][2] * G[1][0] + Fq[1][2] * G[1][1] + Fq[2][2] * G[1][2] -
                  (Fq[0][1] * G[2][0] + Fq[1][1] * G[2][1] + Fq[2][1] * G[2][2]);
          cq[1] = Fq[0][0] * G[2][0] + Fq[1][0] * G[2][1] + Fq[2][0] * G[2][2] -
                  (Fq[0][2] * G[0][0] + Fq[1][2] * G[0][1] + Fq[2][2] * G[0][2]);
          cq[2] = Fq[0][1] * G[0][0] + Fq[1][1] * G[0][1] + Fq[2][1] * G[0][2] -
                  (Fq[0][0] * G[1][0] + Fq[1][0] * G[1][1] + Fq[2][0] * G[1][2]);
#pragma unroll
          for (int m = 0; m < 3; m++) J[m] = (Fq[m][0] * cq[0] + Fq[m][1] * cq[1] + Fq[m][2] * cq[2]) * rDq;
        }
        if constexpr (DIAG) {
#pragma unroll
          for (int m = 0; m < 3; m++) so_p[1][m] = J[m];
          // alpha* = J.B / B^2 (Sec. 3.2.1); 0 where B vanishes
          const double B2 = (double)Bq[0] * Bq[0] + (double)Bq[1] * Bq[1] + (double)Bq[2] * Bq[2];
          const double JB = (double)J[0] * Bq[0] + (double)J[1] * Bq[1] + (double)J[2] * Bq[2];
          so_p[2][0] = B2 > 0.0 ? JB / B2 : 0.0;
        }
        const T f0 = J[1] * Bq[2] - J[2] * Bq[1];
        const T f1 = J[2] * Bq[0] - J[0] * Bq[2];
        const T f2 = J[0] * Bq[1] - J[1] * Bq[0];
        const T gm = (T)gamma;
        u[0] = gm * f0;
        u[1] = gm * f1;
        u[2] = gm * f2;
        if (STAGE1 && tile_ok) {
          const double F2 = (double)f0 * f0 + (double)f1 * f1 + (double)f2 * f2;
          const double B2 = (double)Bq[0] * Bq[0] + (double)Bq[1] * Bq[1] + (double)Bq[2] * Bq[2];
          acc_R2 += Dq * F2;
          if (B2 > tau_B2) {
            const double B4 = B2 * B2;
            if (F2 * xi_B4 > xi_F2 * B4 || F2 != F2) {
              xi_F2 = F2;
              xi_B4 = B4;
              xi_B2 = B2;
            }
          } else {
            acc_null += 1.0;
          }
        }
      }
      if constexpr (STAGE1) {
        const double sc = (diag_only && a.u_det_scale != 0.0) ? Dq * a.u_det_scale : 1.0;
#pragma unroll
        for (int m = 0; m < 3; m++) {
          so_k[m] = diag_only ? (T)((double)u[m] * sc) : u[m];
          so_y[m] = ycq[m];
        }
      } else if constexpr (S == 2) {
        // y_3 = x_n + dt (a_31 k_1 + a_32 k_2), from the own node's x_n and k_1 of plane q
#pragma unroll
        for (int m = 0; m < 3; m++) {
          const double d3 = fma(dt * CK::a[2][1], (double)u[m], (dt * CK::a[2][0]) * (double)kq[m]);
          so_y[m] = xq[m] + d3;
          so_k[m] = u[m];
        }
      } else if constexpr (S == 3) {
        // d_4 = dt (a_41 k_1 + a_42 k_2 + a_43 k_3)
#pragma unroll
        for (int m = 0; m < 3; m++) {
          double d4 = (dt * CK::a[3][0]) * (double)pk[0][m];
          d4 = fma(dt * CK::a[3][1], (double)pk[1][m], d4);
          d4 = fma(dt * CK::a[3][2], (double)u[m], d4);
          so_k[m] = u[m];
          so_s[0][m] = (T)d4;
        }
      } else if constexpr (S == 4) {
        // y_5 = x_n + d_5, and the partial sums of k_1..k_4 the last two stages need
        // (b5_2 = b4_2 = 0: k_2 enters neither X nor E)
#pragma unroll
        for (int m = 0; m < 3; m++) {
          const double k1 = pk[0][m], k2 = pk[1][m], k3 = pk[2][m], k4 = u[m];
          double d5 = (dt * CK::a[4][0]) * k1;
          d5 = fma(dt * CK::a[4][1], k2, d5);
          d5 = fma(dt * CK::a[4][2], k3, d5);
          d5 = fma(dt * CK::a[4][3], k4, d5);
          double p6 = (dt * CK::a[5][0]) * k1;
          p6 = fma(dt * CK::a[5][1], k2, p6);
          p6 = fma(dt * CK::a[5][2], k3, p6);
          p6 = fma(dt * CK::a[5][3], k4, p6);
          double xs = (dt * CK::b5[0]) * k1;
          xs = fma(dt * CK::b5[2], k3, xs);
          xs = fma(dt * CK::b5[3], k4, xs);
          double es = (dt * (CK::b5[0] - CK::b4[0])) * k1;
          es = fma(dt * (CK::b5[2] - CK::b4[2]), k3, es);
          es = fma(dt * (CK::b5[3] - CK::b4[3]), k4, es);
          so_y[m] = xq[m] + d5;
          so_s[0][m] = (T)p6;
          so_s[1][m] = (T)xs;
          so_s[2][m] = (T)es;
        }
      } else if constexpr (S == 5) {
#pragma unroll
        for (int m = 0; m < 3; m++) {
          so_s[0][m] = (T)fma(dt * CK::a[5][4], (double)u[m], (double)ps[0][m]);
          so_s[2][m] = (T)fma(dt * (CK::b5[4] - CK::b4[4]), (double)u[m], (double)ps[1][m]);
        }
      } else {
        // x_{n+1} = x_n + (X + dt b5_6 k_6);  error E + dt (b5_6 - b4_6) k_6
#pragma unroll
        for (int m = 0; m < 3; m++) {
          so_y[m] = xq[m] + fma(dt * CK::b5[5], (double)u[m], (double)ps[0][m]);
          const double e = fma(dt * (CK::b5[5] - CK::b4[5]), (double)u[m], (double)ps[1][m]);
          const double err = tile_ok ? fabs(e) : 0.0;
          acc_lam = (err > acc_lam || err != err) ? err : acc_lam;
        }
      }
    }
    load_point(p);  // output node of the next plane step
    if constexpr (NNN) load_window(hi + 1);
    store_plane(q, qout);
    __syncthreads();

#pragma unroll
    for (int m = 0; m < 3; m++) {
      Bqm[m] = Bq[m];
      Bq[m] = Bp[m];
      Fzq[m] = Fzp[m];
    }
    rDq = rDp;
    Dq = Dp;
    kap_q = kap_p;
  }

  // ---- workgroup reductions -> partial records -----------------------------------------
  const int wave = tid >> 6, lane = tid & 63;
  if (STAGE1) {
    const double acc_xi = sqrt(xi_F2) / xi_B2;
    const double e = wave_sum(acc_E), r2 = wave_sum(acc_R2), xi = wave_max(acc_xi), mn = wave_min(acc_min),
                 nl = wave_sum(acc_null), cc = wave_sum(acc_conc);
    if (lane == 0) {
      red[wave][0] = e;
      red[wave][1] = r2;
      red[wave][2] = xi;
      red[wave][3] = mn;
      red[wave][4] = nl;
      red[wave][5] = cc;
    }
    __syncthreads();
    if (tid == 0) {
      double E = 0, R = 0, X = 0, M = INFINITY, Z = 0, Cc = 0;
      for (int w = 0; w < NTHREADS / 64; w++) {
        E += red[w][0];
        R += red[w][1];
        X = (red[w][2] > X || red[w][2] != red[w][2]) ? red[w][2] : X;
        M = (red[w][3] < M || red[w][3] != red[w][3]) ? red[w][3] : M;
        Z += red[w][4];
        Cc += red[w][5];
      }
      double* pp = a.part + (long long)blockIdx.x * NPART;
      pp[0] = E;
      pp[1] = R;
      pp[2] = X;
      pp[3] = M;
      pp[4] = Z;
      pp[5] = Cc;
    }
  }
  if (LAST) {
    const double l = wave_max(acc_lam);
    if (lane == 0) red[wave][5] = l;
    __syncthreads();
    if (tid == 0) {
      double L = 0;
      for (int w = 0; w < NTHREADS / 64; w++) L = (red[w][5] > L || red[w][5] != red[w][5]) ? red[w][5] : L;
      a.lam_part[blockIdx.x] = L;
    }
  }
}

template <bool MIXED, bool XYP, bool NNN = false>
hipError_t launch_stage_t(int s, const SweepArgs& a, hipStream_t st) {
  const dim3 grid(a.g.nblocks), block(NTHREADS);
  switch (s) {
    case 1: hipLaunchKernelGGL((stage_kernel<1, MIXED, XYP, false, false, NNN>), grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL((stage_kernel<2, MIXED, XYP, false, false, NNN>), grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL((stage_kernel<3, MIXED, XYP, false, false, NNN>), grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL((stage_kernel<4, MIXED, XYP, false, false, NNN>), grid, block, 0, st, a); break;
    case 5: hipLaunchKernelGGL((stage_kernel<5, MIXED, XYP, false, false, NNN>), grid, block, 0, st, a); break;
    case 6: hipLaunchKernelGGL((stage_kernel<6, MIXED, XYP, false, false, NNN>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// the forward replay of the reverse pass (FP64): stages 4 and 6 also store their input
template <bool XYP>
hipError_t launch_stage_rec_t(int s, const SweepArgs& a, hipStream_t st) {
  const dim3 grid(a.g.nblocks), block(NTHREADS);
  switch (s) {
    case 4: hipLaunchKernelGGL((stage_kernel<4, false, XYP, false, true>), grid, block, 0, st, a); break;
    case 6: hipLaunchKernelGGL((stage_kernel<6, false, XYP, false, true>), grid, block, 0, st, a); break;
    default: return launch_stage_t<false, XYP>(s, a, st);
  }
  return hipGetLastError();
}

template <bool XYP, bool NNN>
hipError_t launch_diagnostics_t(const SweepArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((stage_kernel<1, false, XYP, true, false, NNN>), dim3(a.g.nblocks), dim3(NTHREADS), 0, st, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_stage(int s, bool mixed, const SweepArgs& a, hipStream_t st) {
  const bool xyp = (a.g.bc[0] == BC_PERIODIC && a.g.bc[1] == BC_PERIODIC);
  if (a.g.curl == CURL_NNN) {
    if (mixed) return hipErrorInvalidValue;
    return xyp ? launch_stage_t<false, true, true>(s, a, st) : launch_stage_t<false, false, true>(s, a, st);
  }
  if (mixed) return xyp ? launch_stage_t<true, true>(s, a, st) : launch_stage_t<true, false>(s, a, st);
  return xyp ? launch_stage_t<false, true>(s, a, st) : launch_stage_t<false, false>(s, a, st);
}

hipError_t launch_stage_rec(int s, const SweepArgs& a, hipStream_t st) {
  if (a.g.curl == CURL_NNN) return hipErrorInvalidValue;
  const bool xyp = (a.g.bc[0] == BC_PERIODIC && a.g.bc[1] == BC_PERIODIC);
  return xyp ? launch_stage_rec_t<true>(s, a, st) : launch_stage_rec_t<false>(s, a, st);
}

hipError_t launch_diagnostics(const SweepArgs& a, hipStream_t st) {
  const bool xyp = (a.g.bc[0] == BC_PERIODIC && a.g.bc[1] == BC_PERIODIC);
  if (a.g.curl == CURL_NNN)
    return xyp ? launch_diagnostics_t<true, true>(a, st) : launch_diagnostics_t<false, true>(a, st);
  return xyp ? launch_diagnostics_t<true, false>(a, st) : launch_diagnostics_t<false, false>(a, st);
}

}  // namespace relax
