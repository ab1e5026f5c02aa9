// stage.hip -- the fused Runge-Kutta stage sweep of the mimetic magneto-frictional step.
//
// One launch evaluates, for every node, the right-hand side u = gamma J x B of the
// Lagrangian relaxation (eq. "magneto friction") at the stage input
//     y_s = x_n + dt sum_{j<s} a_sj k_j                  (Cash-Karp RK5(4), Sec. 2.4)
// and stores k_s = u(y_s).  Stage 1 also reduces the diagnostics of x_n (E_M with the
// face weights zeta, eq. "magnetic energy"; xi = max |J x B| / B^2; R2; min Delta);
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
// Data flow: a workgroup owns a 64 x 4 (x, y) tile and marches up a z-chunk.  Each plane
// of the stage input y (tile + 2-node halo, FP64) is assembled from x_n and the k_j into an
// LDS ring of three planes; F', det F' and B are formed on the tile + 1-node halo into an
// LDS ring of three B planes; the current, force and velocity are formed on the tile one
// plane behind.  The global loads of the next plane are issued before the current plane
// is computed and committed to LDS after it.
#include <type_traits>

#include "relax_device.h"

// k vectors of an FP64 stage input loaded before the field computation (the rest after it)
#ifndef RELAX_FP64_PHASE_A
#define RELAX_FP64_PHASE_A 5
#endif

namespace relax {
namespace {

__device__ __forceinline__ int floordiv(int a, int n) { return a >= 0 ? a / n : -((-a + n - 1) / n); }
__device__ __forceinline__ int mod3(int p) { return ((p % 3) + 3) % 3; }

struct AxisIdx {
  int i;   // in-range index
  int w;   // periods wrapped
  bool ok;
};

__device__ __forceinline__ AxisIdx resolve(int v, int n, int bc) {
  AxisIdx r;
  if (bc == BC_PERIODIC) {
    r.w = floordiv(v, n);
    r.i = v - r.w * n;
    r.ok = true;
  } else {
    r.w = 0;
    r.i = v;
    r.ok = (v >= 0 && v < n);
  }
  return r;
}

// logical tile of this workgroup; consecutive logical tiles share an XCD (the hardware
// hands workgroup b to XCD b mod 8), so neighbouring tiles reuse each other's halos in L2
__device__ __forceinline__ int logical_block(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = bid & 7, j = bid >> 3;
  return xcd * q + (xcd < r ? xcd : r) + j;
}

template <typename T>
__device__ __forceinline__ T det3(const T F[3][3]) {
  return F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
         F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
}

// 1/d by the hardware estimate and two Newton steps (d is a positive normal number here;
// d <= 0 means a folded cell, which the step control reports from det F itself)
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

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

// S: stage 1..6.  MIXED: k and B0 in FP32 and the stencil past F' in FP32.  XYP: x and y
// both periodic (no line-tied rows or range checks in x and y).
template <int S, bool MIXED, bool XYP>
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(2))) void stage_kernel(SweepArgs a) {
  using T = typename std::conditional<MIXED, float, double>::type;
  constexpr bool STAGE1 = (S == 1);
  constexpr bool LAST = (S == 6);
  constexpr int NK = (S > 1) ? S - 1 : 1;                     // k vectors in the stage input
  constexpr int NP2 = (RY2 * RX2 + NTHREADS - 1) / NTHREADS;  // stage-input points per thread
  constexpr int NP1 = (RY1 * RX1 + NTHREADS - 1) / NTHREADS;  // field points per thread

  Control* ctl = a.ctl;
  const bool diag_only = (a.diag_only != 0);
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
  // dt a_sj folded into one coefficient per k_j
  double cka[NK];
#pragma unroll
  for (int j = 0; j < NK; j++) cka[j] = (S > 1) ? dt * CK::a[S - 1][j] : 0.0;

  const Geometry& g = a.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const long long N = g.N;
  const int bcx = XYP ? BC_PERIODIC : g.bc[0];
  const int bcy = XYP ? BC_PERIODIC : g.bc[1];
  const int bcz = g.bc[2];
  const double inv8h3 = g.inv8h3;

  const int lb = logical_block(blockIdx.x, g.nblocks);
  const int tile_x = lb % g.tiles[0];
  const int tile_y = (lb / g.tiles[0]) % g.tiles[1];
  const int chunk = lb / (g.tiles[0] * g.tiles[1]);
  const int i0 = tile_x * TX, j0 = tile_y * TY;
  const int z0 = chunk * g.tz;
  const int z1 = min(z0 + g.tz, nz);

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;

  __shared__ double ys[3][3][RY2 * RX2];  // stage input, tile + 2-node halo, ring of 3 planes
  __shared__ T bs[3][3][RY1 * RX1];       // pulled-back field, tile + 1-node halo, ring of 3
  __shared__ double red[NTHREADS / 64][NPART];

  const double* __restrict__ xn = a.x[cur];
  const T* __restrict__ b0p = static_cast<const T*>(a.B0);
  const long long nxy = (long long)nx * ny;

  // ---- per-thread index tables: the (x, y) part of every address is the same on all planes
  int w2xy[NP2];  // stage-input window point -> flat (x, y) index, -1 off the grid
  int w2w[NP2];   // its periodic wraps: x in the low 16 bits, y in the high 16 bits (signed)
#pragma unroll
  for (int r = 0; r < NP2; r++) {
    const int e = tid + r * NTHREADS;
    const int row = e / RX2, col = e - row * RX2;
    const AxisIdx rx = resolve(i0 + col - 2, nx, bcx);
    const AxisIdx ry = resolve(j0 + row - 2, ny, bcy);
    w2xy[r] = (e < RY2 * RX2 && rx.ok && ry.ok) ? ry.i * nx + rx.i : -1;
    w2w[r] = (ry.w << 16) + (rx.w & 0xffff);
  }
  // field point e: e < NTHREADS is the tile point of thread e; the rest is the halo ring
  int f1xy[NP1], f1r[NP1], f1c[NP1];
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
    f1xy[r] = (e < RY1 * RX1 && rx.ok && ry.ok) ? ry.i * nx + rx.i : -1;
    f1r[r] = (e < RY1 * RX1) ? r1 : -1;
    f1c[r] = c1;
  }

  // ---- stage-input plane: global loads into registers (issue), then y -> LDS (commit) ----
  // Phase A (x_n and the first NA k_j) is issued before the field computation of the
  // current plane; with FP64 stage vectors the remaining NB k_j (phase B) are issued after
  // phase A has been folded into a partial sum, which bounds the registers held in flight.
  constexpr int NA = MIXED ? NK : (NK < RELAX_FP64_PHASE_A ? NK : RELAX_FP64_PHASE_A);
  constexpr int NB = (S > 1) ? (S - 1) - NA : 0;
  constexpr int NBA = NB > 0 ? NB : 1;
  double px[NP2][3];
  T pk[NK][NP2][3];
  T pkb[NBA][NP2][3];
  double yacc[NP2][3];
  auto issue_a = [&](int pz) {
    const long long zo = resolve(pz, nz, bcz).i * nxy;
#pragma unroll
    for (int r = 0; r < NP2; r++) {
      if (w2xy[r] >= 0) {
        const unsigned o = (unsigned)w2xy[r];
#pragma unroll
        for (int m = 0; m < 3; m++) px[r][m] = (xn + zo + m * N)[o];
        if constexpr (S > 1) {
#pragma unroll
          for (int j = 0; j < NA; j++) {
            const T* __restrict__ kj = static_cast<const T*>(a.k[j]) + zo;
#pragma unroll
            for (int m = 0; m < 3; m++) pk[j][r][m] = (kj + m * N)[o];
          }
        }
      }
    }
  };
  auto fold_a = [&]() {
#pragma unroll
    for (int r = 0; r < NP2; r++)
#pragma unroll
      for (int m = 0; m < 3; m++) {
        double y = px[r][m];
        if constexpr (S > 1) {
#pragma unroll
          for (int j = 0; j < NA; j++) y = fma(cka[j], (double)pk[j][r][m], y);
        }
        yacc[r][m] = y;
      }
  };
  auto issue_b = [&](int pz) {
    if constexpr (NB > 0) {
      const long long zo = resolve(pz, nz, bcz).i * nxy;
#pragma unroll
      for (int r = 0; r < NP2; r++) {
        if (w2xy[r] >= 0) {
          const unsigned o = (unsigned)w2xy[r];
#pragma unroll
          for (int j = 0; j < NB; j++) {
            const T* __restrict__ kj = static_cast<const T*>(a.k[NA + j]) + zo;
#pragma unroll
            for (int m = 0; m < 3; m++) pkb[j][r][m] = (kj + m * N)[o];
          }
        }
      }
    }
  };
  auto commit_plane = [&](int pz) {
    const AxisIdx rz = resolve(pz, nz, bcz);
    const int slot = mod3(pz);
    const double shz = rz.w * g.period[2];
    if constexpr (NB == 0) fold_a();
#pragma unroll
    for (int r = 0; r < NP2; r++) {
      const int e = tid + r * NTHREADS;
      if (e < RY2 * RX2) {
        double v[3] = {0.0, 0.0, 0.0};
        if (w2xy[r] >= 0) {
#pragma unroll
          for (int m = 0; m < 3; m++) {
            double y = yacc[r][m];
            if constexpr (NB > 0) {
#pragma unroll
              for (int j = 0; j < NB; j++) y = fma(cka[NA + j], (double)pkb[j][r][m], y);
            }
            v[m] = y;
          }
          v[0] += (double)(short)(w2w[r] & 0xffff) * g.period[0];
          v[1] += (double)(w2w[r] >> 16) * g.period[1];
          v[2] += shz;
        }
#pragma unroll
        for (int m = 0; m < 3; m++) ys[slot][m][e] = v[m];
      }
    }
  };
  auto issue_b0 = [&](int p, T (&dst)[NP1][3]) {
    const long long zo = resolve(p, nz, bcz).i * nxy;
#pragma unroll
    for (int r = 0; r < NP1; r++) {
      if (f1xy[r] >= 0) {
        const unsigned o = (unsigned)f1xy[r];
#pragma unroll
        for (int m = 0; m < 3; m++) dst[r][m] = (b0p + zo + m * N)[o];
      } else {
#pragma unroll
        for (int m = 0; m < 3; m++) dst[r][m] = T(0);
      }
    }
  };

  // ---- unscaled Jacobian at a window point (r, c in stage-input window coordinates) -----
  auto jac_xy = [&](int r, int c, int p, int gi, int gj, double F[3][3]) {
    const int o = r * RX2 + c;
    const int sp = mod3(p);
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
    const int o = r * RX2 + c;
    const int sp = mod3(p);
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
    if (bcz == BC_PERIODIC || (p > 0 && p < nz - 1)) {
      const int sa = mod3(p + 1), sb = mod3(p - 1);
#pragma unroll
      for (int m = 0; m < 3; m++) F[m][2] = ys[sa][m][o] - ys[sb][m][o];
    } else if (p == 0) {
#pragma unroll
      for (int m = 0; m < 3; m++) F[m][2] = -3.0 * ys[0][m][o] + 4.0 * ys[1][m][o] - ys[2][m][o];
    } else {
      const int s0 = mod3(p), s1 = mod3(p - 1), s2 = mod3(p - 2);
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

  // tile point owned by this thread
  const int gi_t = i0 + tx, gj_t = j0 + ty;
  const bool tile_ok = (gi_t < nx) && (gj_t < ny);
  const bool face_xy = !XYP && ((bcx == BC_LINE_TIED && (gi_t == 0 || gi_t == nx - 1)) ||
                                (bcy == BC_LINE_TIED && (gj_t == 0 || gj_t == ny - 1)));

  // reductions
  double acc_E = 0.0, acc_R2 = 0.0, acc_xi = 0.0, acc_min = INFINITY, acc_null = 0.0, acc_lam = 0.0;

  // one plane step: field B(p) on the tile + halo (tile point's F' -> Fo, 1/det F' -> rDo,
  // det F -> Do), then u at plane q = p - 1 from Fi / rDi / Di (the previous plane's)
  auto plane = [&](int p, const double (&Fzi)[3], double rDi, double Di, double (&Fzo)[3], double& rDo,
                   double& Do, T (&b0use)[NP1][3]) {
    // the per-lane offsets are made opaque here so that the compiler recomputes addresses
    // per plane instead of keeping one hoisted 64-bit address per array, component and slot
#pragma unroll
    for (int r = 0; r < NP2; r++) asm volatile("" : "+v"(w2xy[r]));
#pragma unroll
    for (int r = 0; r < NP1; r++) asm volatile("" : "+v"(f1xy[r]));
    const int q = p - 1;
    const bool out_here = (q >= z0 && q < z1 && tile_ok);
    const long long out_zo = resolve(q, nz, bcz).i * nxy;     // uniform
    unsigned out_o = out_here ? (unsigned)(gj_t * nx + gi_t) : 0u;
    asm volatile("" : "+v"(out_o));

    // 1. prefetch phase A of the next stage-input plane
    const bool pre_plane = (p + 1 <= pb1) && (need_hi(p + 1) > need_hi(p));
    const int pre_z = need_hi(p) + 1;
    if (pre_plane) issue_a(pre_z);

    // 2. F', det F' and B on the tile + 1-node halo of plane p
    if (p <= pb1) {
      const int sp = mod3(p);
      const long long zo = resolve(p, nz, bcz).i * nxy;
#pragma unroll
      for (int r = 0; r < NP1; r++) {
        __builtin_amdgcn_sched_barrier(0);  // one field point at a time: bounds live temporaries
        if (f1r[r] >= 0) {
          const int r1 = f1r[r], c1 = f1c[r];
          const int gi = i0 + c1 - 1, gj = j0 + r1 - 1;
          T B[3] = {T(0), T(0), T(0)};
          if (f1xy[r] >= 0) {
            double F[3][3];
            jacobian(r1 + 1, c1 + 1, p, gi, gj, F);
            const double D = det3(F);
            const double rD = rcp_nr(D);
            const T q0 = b0use[r][0], q1 = b0use[r][1], q2 = b0use[r][2];
            if constexpr (MIXED) {
              const float fi = (float)rD;
#pragma unroll
              for (int m = 0; m < 3; m++)
                B[m] = ((float)F[m][0] * q0 + (float)F[m][1] * q1 + (float)F[m][2] * q2) * fi;
            } else {
#pragma unroll
              for (int m = 0; m < 3; m++) B[m] = (F[m][0] * q0 + F[m][1] * q1 + F[m][2] * q2) * rD;
            }
            if (r == 0) {  // this thread's own tile point
#pragma unroll
              for (int m = 0; m < 3; m++) Fzo[m] = F[m][2];
              rDo = rD;
              Do = D * inv8h3;
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
                acc_E += zeta * (Bd[0] * Bd[0] + Bd[1] * Bd[1] + Bd[2] * Bd[2]) * Do;
                acc_min = (Do < acc_min || Do != Do) ? Do : acc_min;
                if (record_ck) {
                  double* ck = a.ckpt + ck_slot * 3 * N;
                  const unsigned o = (unsigned)f1xy[r];
#pragma unroll
                  for (int m = 0; m < 3; m++) (ck + zo + m * N)[o] = (xn + zo + m * N)[o];
                }
              }
            }
          }
#pragma unroll
          for (int m = 0; m < 3; m++) bs[sp][m][r1 * RX1 + c1] = B[m];
        }
      }
    }
    // x and y columns of the tile point's Jacobian at plane q, read before the barrier: the
    // commit at the end of this step reuses plane q's ring slot
    double Fxy[3][3];
    if (out_here) jac_xy(ty + 2, tx + 2, q, gi_t, gj_t, Fxy);
    __syncthreads();

    // 3. current, force and velocity on the tile of plane q = p - 1
    // (stage 6 first fetches the output node's x_n and k_j)
    double sx[3] = {0, 0, 0};
    T sk[4][3];
    if constexpr (LAST) {
      if (out_here && !diag_only) {
#pragma unroll
        for (int m = 0; m < 3; m++) {
          const long long b = out_zo + m * N;
          sx[m] = (xn + b)[out_o];
          sk[0][m] = (static_cast<const T*>(a.k[0]) + b)[out_o];
          sk[1][m] = (static_cast<const T*>(a.k[2]) + b)[out_o];
          sk[2][m] = (static_cast<const T*>(a.k[3]) + b)[out_o];
          sk[3][m] = (static_cast<const T*>(a.k[4]) + b)[out_o];
        }
      }
    }
    // fold phase A, issue phase B of the next plane and B0 of the next field plane (the
    // previous B0 registers were consumed above)
    if constexpr (NB > 0) {
      if (pre_plane) {
        fold_a();
        issue_b(pre_z);
      }
    }
    if (p + 1 <= pb1) issue_b0(p + 1, b0use);
    if (out_here) {
      const bool face = face_xy || (bcz == BC_LINE_TIED && (q == 0 || q == nz - 1));
      T u[3] = {T(0), T(0), T(0)};
      if (!face) {
        const int o = (ty + 1) * RX1 + (tx + 1);
        const int sq = mod3(q), sm = mod3(q - 1), spl = mod3(q + 1);
        T G[3][3];  // G'[a][m] = B_m(n + e_a) - B_m(n - e_a)
#pragma unroll
        for (int m = 0; m < 3; m++) {
          G[0][m] = bs[sq][m][o + 1] - bs[sq][m][o - 1];
          G[1][m] = bs[sq][m][o + RX1] - bs[sq][m][o - RX1];
          G[2][m] = bs[spl][m][o] - bs[sm][m][o];
        }
        // the tile point's Jacobian at plane q: x and y columns recomputed from the stage
        // input before the barrier, z column carried from the previous field step
        T Fq[3][3];
#pragma unroll
        for (int m = 0; m < 3; m++) {
          Fq[m][0] = (T)Fxy[m][0];
          Fq[m][1] = (T)Fxy[m][1];
          Fq[m][2] = (T)Fzi[m];
        }
        // c'_q = (F' e_b) . G'_a - (F' e_a) . G'_b, (a, b, q) = (y, z, x), (z, x, y), (x, y, z)
        T cq[3];
        cq[0] = Fq[0][2] * G[1][0] + Fq[1][2] * G[1][1] + Fq[2][2] * G[1][2] -
                (Fq[0][1] * G[2][0] + Fq[1][1] * G[2][1] + Fq[2][1] * G[2][2]);
        cq[1] = Fq[0][0] * G[2][0] + Fq[1][0] * G[2][1] + Fq[2][0] * G[2][2] -
                (Fq[0][2] * G[0][0] + Fq[1][2] * G[0][1] + Fq[2][2] * G[0][2]);
        cq[2] = Fq[0][1] * G[0][0] + Fq[1][1] * G[0][1] + Fq[2][1] * G[0][2] -
                (Fq[0][0] * G[1][0] + Fq[1][0] * G[1][1] + Fq[2][0] * G[1][2]);
        const T iD = (T)rDi;
        T J[3];
#pragma unroll
        for (int m = 0; m < 3; m++) J[m] = (Fq[m][0] * cq[0] + Fq[m][1] * cq[1] + Fq[m][2] * cq[2]) * iD;
        const T Bq0 = bs[sq][0][o], Bq1 = bs[sq][1][o], Bq2 = bs[sq][2][o];
        const T f0 = J[1] * Bq2 - J[2] * Bq1;
        const T f1 = J[2] * Bq0 - J[0] * Bq2;
        const T f2 = J[0] * Bq1 - J[1] * Bq0;
        const T gm = (T)gamma;
        u[0] = gm * f0;
        u[1] = gm * f1;
        u[2] = gm * f2;
        if (STAGE1) {
          const double F2 = (double)f0 * f0 + (double)f1 * f1 + (double)f2 * f2;
          const double B2 = (double)Bq0 * Bq0 + (double)Bq1 * Bq1 + (double)Bq2 * Bq2;
          acc_R2 += Di * F2;
          if (B2 > tau_B2) {
            const double ratio = sqrt(F2) / B2;
            acc_xi = (ratio > acc_xi || ratio != ratio) ? ratio : acc_xi;
          } else {
            acc_null += 1.0;
          }
        }
      }
      if (diag_only) {
        if (a.u_out) {
          const double sc = (a.u_det_scale != 0.0) ? Di * a.u_det_scale : 1.0;
#pragma unroll
          for (int m = 0; m < 3; m++) (a.u_out + out_zo + m * N)[out_o] = (double)u[m] * sc;
        }
      } else {
        if constexpr (!LAST) {
          T* __restrict__ ks = static_cast<T*>(a.k[S - 1]);
#pragma unroll
          for (int m = 0; m < 3; m++) (ks + out_zo + m * N)[out_o] = u[m];
        } else {
          // x_{n+1} = x_n + dt sum b5_s k_s;  err = dt sum (b5_s - b4_s) k_s
          double* __restrict__ xo = a.xout[1 - cur];
#pragma unroll
          for (int m = 0; m < 3; m++) {
            const double v1 = sk[0][m], v3 = sk[1][m], v4 = sk[2][m], v5 = sk[3][m], v6 = (double)u[m];
            const double s5 = CK::b5[0] * v1 + CK::b5[2] * v3 + CK::b5[3] * v4 + CK::b5[5] * v6;
            const double se = (CK::b5[0] - CK::b4[0]) * v1 + (CK::b5[2] - CK::b4[2]) * v3 +
                              (CK::b5[3] - CK::b4[3]) * v4 + (CK::b5[4] - CK::b4[4]) * v5 +
                              (CK::b5[5] - CK::b4[5]) * v6;
            (xo + out_zo + m * N)[out_o] = sx[m] + dt * s5;
            const double err = fabs(dt * se);
            acc_lam = (err > acc_lam || err != err) ? err : acc_lam;
          }
        }
      }
    }

    // 4. commit the prefetched plane (its ring slot held the plane B(p) no longer needs)
    if (pre_plane) commit_plane(pre_z);
    __syncthreads();
  };

  // prologue: the first window, synchronously; B0 of the first plane
  for (int pz = need_lo(pb0); pz <= need_hi(pb0); pz++) {
    issue_a(pz);
    if constexpr (NB > 0) {
      fold_a();
      issue_b(pz);
    }
    commit_plane(pz);
  }
  double Fzprev[3] = {0, 0, 0}, Fzcur[3] = {0, 0, 0};
  double rDprev = 0.0, rDcur = 0.0, Dprev = 0.0, Dcur = 0.0;
  T b0reg[NP1][3];
  issue_b0(pb0, b0reg);
  __syncthreads();
  for (int p = pb0; p <= pb1 + 1; p++) {
    plane(p, Fzprev, rDprev, Dprev, Fzcur, rDcur, Dcur, b0reg);
#pragma unroll
    for (int m = 0; m < 3; m++) Fzprev[m] = Fzcur[m];
    rDprev = rDcur;
    Dprev = Dcur;
  }

  // ---- workgroup reductions -> partial records -----------------------------------------
  const int wave = tid >> 6, lane = tid & 63;
  if (STAGE1) {
    const double e = wave_sum(acc_E), r2 = wave_sum(acc_R2), xi = wave_max(acc_xi), mn = wave_min(acc_min),
                 nl = wave_sum(acc_null);
    if (lane == 0) {
      red[wave][0] = e;
      red[wave][1] = r2;
      red[wave][2] = xi;
      red[wave][3] = mn;
      red[wave][4] = nl;
    }
    __syncthreads();
    if (tid == 0) {
      double E = 0, R = 0, X = 0, M = INFINITY, Z = 0;
      for (int w = 0; w < NTHREADS / 64; w++) {
        E += red[w][0];
        R += red[w][1];
        X = (red[w][2] > X || red[w][2] != red[w][2]) ? red[w][2] : X;
        M = (red[w][3] < M || red[w][3] != red[w][3]) ? red[w][3] : M;
        Z += red[w][4];
      }
      double* pp = a.part + (long long)blockIdx.x * NPART;
      pp[0] = E;
      pp[1] = R;
      pp[2] = X;
      pp[3] = M;
      pp[4] = Z;
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

template <bool MIXED, bool XYP>
hipError_t launch_stage_t(int s, const SweepArgs& a, hipStream_t st) {
  const dim3 grid(a.g.nblocks), block(NTHREADS);
  switch (s) {
    case 1: hipLaunchKernelGGL((stage_kernel<1, MIXED, XYP>), grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL((stage_kernel<2, MIXED, XYP>), grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL((stage_kernel<3, MIXED, XYP>), grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL((stage_kernel<4, MIXED, XYP>), grid, block, 0, st, a); break;
    case 5: hipLaunchKernelGGL((stage_kernel<5, MIXED, XYP>), grid, block, 0, st, a); break;
    case 6: hipLaunchKernelGGL((stage_kernel<6, MIXED, XYP>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_stage(int s, bool mixed, const SweepArgs& a, hipStream_t st) {
  const bool xyp = (a.g.bc[0] == BC_PERIODIC && a.g.bc[1] == BC_PERIODIC);
  if (mixed) return xyp ? launch_stage_t<true, true>(s, a, st) : launch_stage_t<true, false>(s, a, st);
  return xyp ? launch_stage_t<false, true>(s, a, st) : launch_stage_t<false, false>(s, a, st);
}

hipError_t launch_diagnostics(const SweepArgs& a, hipStream_t st) {
  const bool xyp = (a.g.bc[0] == BC_PERIODIC && a.g.bc[1] == BC_PERIODIC);
  if (xyp)
    hipLaunchKernelGGL((stage_kernel<1, false, true>), dim3(a.g.nblocks), dim3(NTHREADS), 0, st, a);
  else
    hipLaunchKernelGGL((stage_kernel<1, false, false>), dim3(a.g.nblocks), dim3(NTHREADS), 0, st, a);
  return hipGetLastError();
}

}  // namespace relax
