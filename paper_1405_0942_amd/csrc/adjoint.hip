// adjoint.hip -- reverse-mode sweeps of the relaxation step (the transpose of stage.hip).
//
// Forward, per node n (unscaled differences, see stage.hip):
//   F'(n) = D y,  D' = det F',  rD = 1/D',  B = F' B0'' rD,
//   G'_a = B(n+e_a) - B(n-e_a),  c'_q = (F' e_b).G'_a - (F' e_a).G'_b,  w = c' rD,
//   J = F' w,  f = J x B,  u = gamma f (zero on line-tied faces).
// Reverse, given the cotangent ubar of u:
//   fbar = gamma ubar,  Jbar = B x fbar,  Bbar += fbar x J,
//   wbar = F'^T Jbar,   Fbar' += Jbar w^T,  cbar' = rD wbar,  rDbar += wbar . c',
//   Gbar'_x = cbar'_z F'_y - cbar'_y F'_z (and cyclic)  [F'_a = column a],
//   Fbar'_b += cbar'_q G'_a,  Fbar'_a -= cbar'_q G'_b,
//   Bbar(m) += sum_a Gbar'_a(m - e_a) - Gbar'_a(m + e_a)       (transpose of G'),
//   pull-back: Fbar' += (rD Bbar) B0''^T,  B0bar'' += F'^T Bbar rD,  rDbar += Bbar . F'B0'',
//   Dbar' = -rD^2 rDbar,  Fbar' += Dbar' cof(F'),
//   ybar = D^T Fbar'                                           (transpose of the differences).
// Gbar'(n) needs only F', rD, B and ubar at n, so Bbar(m) needs the stage input on a 2-node
// halo of m, the same footprint as the forward sweep.  adj_field_kernel forms Fbar' (9 values
// per node) and accumulates B0bar''; adj_gather_kernel applies D^T and, pointwise, assembles
// the cotangent of the previous stage's k (the Runge-Kutta transpose, see below).
//
// Runge-Kutta transpose of one step x_{n+1} = x_n + dt sum_s b5_s k_s, k_s = u(y_s),
// y_s = x_n + dt sum_{j<s} a_sj k_j:
//   kbar_s = dt (b5_s xbar_{n+1} + sum_{t>s} a_ts ybar_t),  ybar_s = (du/dy)(y_s)^T kbar_s,
//   xbar_n = xbar_{n+1} + sum_s ybar_s.
// The stage-6 field sweep scales xbar_{n+1} itself; the gather of stage t writes ybar_t and
// kbar_{t-1}, which the field sweep of stage t - 1 reads.
//
// Seeds (seed mode of adj_field_kernel): E_M = 1/2 sum zeta |B|^2 det F dV adds kappa D' B to
// Bbar and 1/2 kappa |B|^2 to Dbar' (kappa = zeta dV / (8 hx hy hz)); R2 = 1/2 sum_interior
// det F |f|^2 dV enters through ubar = det F dV f / gamma (read from a buffer) plus
// 1/2 |f|^2 dV / (8 hx hy hz) on Dbar'.
//
// The field sweep is laid out like the forward stage sweep: a 64 x 8 tile marching up a
// z-chunk, the stage input in an LDS ring of three planes (stages 3..6 stencil the stored
// y_s of the step), B in a ring of two planes, Gbar'_x and Gbar'_y in one plane that is
// transposed in-plane as soon as it is formed; buffer loads with masked-off lanes (offsets
// past the record count) issued one plane step ahead, so no divergent branch surrounds a
// memory instruction and the waits are exact.
#include "sweep_common.h"

namespace relax {
namespace {

__device__ __forceinline__ void cross(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

template <int S, bool XYP, bool SEED>
__global__ __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(2))) void adj_field_kernel(AdjArgs a) {
  constexpr bool WK = (!SEED && S == 2);  // the window carries k_1 too
  constexpr int NP2 = (RY2 * RX2 + NTHREADS - 1) / NTHREADS;
  constexpr int NP1 = (RY1 * RX1 + NTHREADS - 1) / NTHREADS;

  const Geometry& g = a.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const long long N = g.N;
  const unsigned nxy = (unsigned)nx * (unsigned)ny;
  const int bcx = XYP ? BC_PERIODIC : g.bc[0];
  const int bcy = XYP ? BC_PERIODIC : g.bc[1];
  const int bcz = g.bc[2];
  const double gamma = a.gamma;

  const double dt = SEED ? 0.0 : *a.dt;
  const double c21 = dt * CK::a[1][0];
  // the cotangent of u: seed buffer, dt b5_6 xbar_{n+1} (stage 6), or the gathered kbar_s
  const bool v_on = !SEED || a.useed != nullptr;
  const double* __restrict__ vsrc = SEED ? (a.useed ? a.useed : a.B0) : (S == 6 ? a.xbar : a.ubar);
  const double cv = (!SEED && S == 6) ? dt * CK::b5[5] : 1.0;
  const double* __restrict__ wsrc = (SEED || S <= 2) ? a.x : a.y[S > 2 ? S - 3 : 0];
  const double* __restrict__ k1p = a.k[0];

  const int lb = logical_block(blockIdx.x, g.nblocks);
  const int tile_x = lb % g.tiles[0];
  const int tile_y = (lb / g.tiles[0]) % g.tiles[1];
  const int chunk = lb / (g.tiles[0] * g.tiles[1]);
  const int i0 = tile_x * TX, j0 = tile_y * TY;
  const int z0 = chunk * g.tz;
  const int z1 = min(z0 + g.tz, nz);
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;

  __shared__ double ys[3][3][RY2 * RX2];  // stage input, ring of 3 planes
  __shared__ double bs[2][3][RY1 * RX1];  // B, ring of 2 planes
  __shared__ double gxy[6][RY1 * RX1];    // Gbar'_x (0..2) and Gbar'_y (3..5) of the newest plane

  auto zload = [&](int pz) {
    if (bcz == BC_PERIODIC) return resolve_near(pz, nz, bcz).i;
    return min(max(pz, 0), nz - 1);
  };

  // index tables (as in the forward sweep)
  unsigned w2e[NP2];
  int w2w[NP2];
#pragma unroll
  for (int r = 0; r < NP2; r++) {
    const int e = tid + r * NTHREADS;
    const int row = e / RX2, col = e - row * RX2;
    const AxisIdx rx = resolve(i0 + col - 2, nx, bcx), ry = resolve(j0 + row - 2, ny, bcy);
    w2e[r] = (e < RY2 * RX2 && rx.ok && ry.ok) ? (unsigned)(ry.i * nx + rx.i) : IE;
    w2w[r] = (ry.w << 16) + (rx.w & 0xffff);
  }
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
  const int gi_t = i0 + tx, gj_t = j0 + ty;
  const bool tile_ok = (gi_t < nx) && (gj_t < ny);
  const unsigned out_e = tile_ok ? (unsigned)(gj_t * nx + gi_t) : IE;

  auto face_at = [&](int gi, int gj, int p) {
    return (bcx == BC_LINE_TIED && (gi == 0 || gi == nx - 1)) || (bcy == BC_LINE_TIED && (gj == 0 || gj == ny - 1)) ||
           (bcz == BC_LINE_TIED && (p == 0 || p == nz - 1));
  };

  // ---- loads, issued one plane step ahead of their use ---------------------------------------
  double wx[NP2][3];
  double wk[WK ? NP2 : 1][3];
  double b0r[NP1][3], vr[NP1][3];
  double bbr[3];  // B0bar'' at the output node
  auto load_window = [&](int pz) {
    const long long zo = (long long)zload(pz) * nxy;
#pragma unroll
    for (int m = 0; m < 3; m++) {
      const auto rs = plane_rsrc(wsrc + m * N + zo, nxy);
#pragma unroll
      for (int r = 0; r < NP2; r++) wx[r][m] = bload<double>(rs, w2e[r]);
    }
    if constexpr (WK) {
#pragma unroll
      for (int m = 0; m < 3; m++) {
        const auto rs = plane_rsrc(k1p + m * N + zo, nxy);
#pragma unroll
        for (int r = 0; r < NP2; r++) wk[r][m] = bload<double>(rs, w2e[r]);
      }
    }
  };
  auto commit_window = [&](int pz) {
    const AxisIdx rz = resolve_near(pz, nz, bcz);
    const int slot = mod3(pz);
    const double shz = rz.w * g.period[2];
#pragma unroll
    for (int r = 0; r < NP2; r++) {
      const int e = tid + r * NTHREADS;
      const bool ok = (w2e[r] != IE);
      double v[3];
#pragma unroll
      for (int m = 0; m < 3; m++) {
        double y = wx[r][m];
        if constexpr (WK) y = fma(c21, wk[r][m], y);
        v[m] = y;
      }
      v[0] += (double)(short)(w2w[r] & 0xffff) * g.period[0];
      v[1] += (double)(w2w[r] >> 16) * g.period[1];
      v[2] += shz;
      if (e < RY2 * RX2) {
#pragma unroll
        for (int m = 0; m < 3; m++) ys[slot][m][e] = ok ? v[m] : 0.0;
      }
    }
  };
  auto load_field = [&](int pz) {
    const long long zo = (long long)zload(pz) * nxy;
#pragma unroll
    for (int m = 0; m < 3; m++) {
      const auto rb = plane_rsrc(a.B0 + m * N + zo, nxy);
      const auto rv = plane_rsrc(vsrc + m * N + zo, nxy);
#pragma unroll
      for (int r = 0; r < NP1; r++) {
        b0r[r][m] = bload<double>(rb, f1e[r]);
        vr[r][m] = bload<double>(rv, v_on ? f1e[r] : IE);
      }
    }
  };
  auto load_point = [&](int pz) {
    const bool on = (pz >= z0 && pz < z1);
    const long long zo = (long long)zload(pz) * nxy;
#pragma unroll
    for (int m = 0; m < 3; m++) bbr[m] = bload<double, CPOL_STREAM>(plane_rsrc(a.B0bar + m * N + zo, nxy), on ? out_e : IE);
  };
  double so_F[9], so_B[3];
#pragma unroll
  for (int i = 0; i < 9; i++) so_F[i] = 0.0;
#pragma unroll
  for (int m = 0; m < 3; m++) so_B[m] = 0.0;
  auto store_point = [&](int qz, bool on) {
    const long long zo = (long long)zload(qz) * nxy;
    const unsigned eo = on ? out_e : IE;
#pragma unroll
    for (int i = 0; i < 9; i++) bstore(plane_rsrc(a.Fbar + i * N + zo, nxy), eo, so_F[i]);
#pragma unroll
    for (int m = 0; m < 3; m++) bstore(plane_rsrc(a.B0bar + m * N + zo, nxy), eo, so_B[m]);
  };

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
    jac_xy(r, c, p, gi, gj, F);
    const int o = r * RX2 + c;
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

  const bool perz = (bcz == BC_PERIODIC);
  const int pb0 = perz ? z0 - 1 : max(z0 - 1, 0);
  const int pb1 = perz ? z1 : min(z1, nz - 1);
  auto need_hi = [&](int p) { return perz ? p + 1 : (p == 0 ? 2 : (p == nz - 1 ? p : p + 1)); };
  auto need_lo = [&](int p) { return perz ? p - 1 : (p == 0 ? 0 : (p == nz - 1 ? p - 2 : p - 1)); };

  // prologue: the first stage-input window, then the loads and (dropped) stores a plane step
  // leaves in flight, in the same order
  int hi = need_hi(pb0);
  for (int pz = need_lo(pb0); pz <= hi; pz++) {
    load_window(pz);
    commit_window(pz);
  }
  __syncthreads();
  load_field(pb0);
  load_window(hi + 1);
  load_point(pb0 - 1);
  store_point(pb0 - 1, false);

  // own-node values carried between plane steps (q = p - 1 is the output plane)
  double Fzq[3] = {0, 0, 0};  // z column of F' at q (the x and y columns are re-read from the ring)
  double rDq = 0.0;
  double ubq[3] = {0, 0, 0}, Bq[3] = {0, 0, 0}, Bqm[3] = {0, 0, 0}, b0q[3] = {0, 0, 0};
  double gzqm[3] = {0, 0, 0}, gzq[3] = {0, 0, 0};  // Gbar'_z at q - 1 and q
  double Bbxyq[3] = {0, 0, 0};                     // in-plane transpose of Gbar' at q
  const int ot = (ty + 1) * RX1 + (tx + 1);

  for (int p = pb0; p <= z1; p++) {
    const int q = p - 1;
    const bool qout = (q >= z0 && q < z1);
    // 1. B, Gbar'_x, Gbar'_y on the tile + 1-node halo of plane p; own-node values
    double Fzp[3] = {0, 0, 0};
    double rDp = 0.0, ubp[3] = {0, 0, 0}, Bp[3] = {0, 0, 0}, b0p[3] = {0, 0, 0}, gzp[3] = {0, 0, 0};
    if (p <= pb1) {
      const int sb = p & 1;
#pragma unroll
      for (int r = 0; r < NP1; r++) {
        __builtin_amdgcn_sched_barrier(0);
        if (f1r[r] >= 0) {
          const int r1 = f1r[r], c1 = f1c[r];
          const int gi = i0 + c1 - 1, gj = j0 + r1 - 1;
          double B[3] = {0, 0, 0}, Gx[3] = {0, 0, 0}, Gy[3] = {0, 0, 0}, Gz[3] = {0, 0, 0}, ub[3] = {0, 0, 0};
          if (f1e[r] != IE) {
            double F[3][3];
            jacobian(r1 + 1, c1 + 1, p, gi, gj, F);
            const double rD = rcp_nr(det3(F));
            const double q0 = b0r[r][0], q1 = b0r[r][1], q2 = b0r[r][2];
#pragma unroll
            for (int m = 0; m < 3; m++) B[m] = (F[m][0] * q0 + F[m][1] * q1 + F[m][2] * q2) * rD;
            if (!face_at(gi, gj, p)) {
#pragma unroll
              for (int m = 0; m < 3; m++) ub[m] = cv * vr[r][m];
              const double fb[3] = {gamma * ub[0], gamma * ub[1], gamma * ub[2]};
              double Jb[3];
              cross(B, fb, Jb);
              double cb[3];  // cbar' = rD F'^T Jbar
#pragma unroll
              for (int n2 = 0; n2 < 3; n2++) cb[n2] = rD * (F[0][n2] * Jb[0] + F[1][n2] * Jb[1] + F[2][n2] * Jb[2]);
#pragma unroll
              for (int m = 0; m < 3; m++) {
                Gx[m] = cb[2] * F[m][1] - cb[1] * F[m][2];
                Gy[m] = cb[0] * F[m][2] - cb[2] * F[m][0];
                Gz[m] = cb[1] * F[m][0] - cb[0] * F[m][1];
              }
            }
            if (r == 0) {
#pragma unroll
              for (int m = 0; m < 3; m++) {
                Fzp[m] = F[m][2];
                ubp[m] = ub[m];
                Bp[m] = B[m];
                b0p[m] = b0r[r][m];
                gzp[m] = Gz[m];
              }
              rDp = rD;
            }
          }
          const int o = r1 * RX1 + c1;
#pragma unroll
          for (int m = 0; m < 3; m++) {
            bs[sb][m][o] = B[m];
            gxy[m][o] = Gx[m];
            gxy[3 + m][o] = Gy[m];
          }
        }
      }
    }
    load_field(p + 1 <= pb1 ? p + 1 : pb1);
    // x and y columns of F' at the own node of plane q, read before the barrier: the commit
    // below reuses plane q's ring slot
    double F[3][3];
    if (qout) {
      jac_xy(ty + 2, tx + 2, q, gi_t, gj_t, F);
#pragma unroll
      for (int m = 0; m < 3; m++) F[m][2] = Fzq[m];
    }
    __syncthreads();

    // 2. commit the stage-input plane field(p + 1) needs; issue the next one
    if (p + 1 <= pb1 && need_hi(p + 1) > hi) {
      hi++;
      commit_window(hi);
    }
    load_window(hi + 1);

    // 3. in-plane transpose of Gbar' at the own node of plane p (used by the next step)
    double Bbxyp[3];
#pragma unroll
    for (int m = 0; m < 3; m++)
      Bbxyp[m] = (gxy[m][ot - 1] - gxy[m][ot + 1]) + (gxy[3 + m][ot - RX1] - gxy[3 + m][ot + RX1]);

    // 4. the transpose at the own node of plane q
    if (qout) {
      const bool interior = !face_at(gi_t, gj_t, q);
      double Bb[3] = {0, 0, 0};
      double Fb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      double rDb = 0.0, Db_direct = 0.0;
      if (interior) {
        const int sq = q & 1;
        double G[3][3];  // G[a][m]
#pragma unroll
        for (int m = 0; m < 3; m++) {
          G[0][m] = bs[sq][m][ot + 1] - bs[sq][m][ot - 1];
          G[1][m] = bs[sq][m][ot + RX1] - bs[sq][m][ot - RX1];
          G[2][m] = Bp[m] - Bqm[m];
        }
        double cq[3];
        cq[0] = F[0][2] * G[1][0] + F[1][2] * G[1][1] + F[2][2] * G[1][2] -
                (F[0][1] * G[2][0] + F[1][1] * G[2][1] + F[2][1] * G[2][2]);
        cq[1] = F[0][0] * G[2][0] + F[1][0] * G[2][1] + F[2][0] * G[2][2] -
                (F[0][2] * G[0][0] + F[1][2] * G[0][1] + F[2][2] * G[0][2]);
        cq[2] = F[0][1] * G[0][0] + F[1][1] * G[0][1] + F[2][1] * G[0][2] -
                (F[0][0] * G[1][0] + F[1][0] * G[1][1] + F[2][0] * G[1][2]);
        const double w[3] = {cq[0] * rDq, cq[1] * rDq, cq[2] * rDq};
        double J[3];
#pragma unroll
        for (int m = 0; m < 3; m++) J[m] = F[m][0] * w[0] + F[m][1] * w[1] + F[m][2] * w[2];
        const double fb[3] = {gamma * ubq[0], gamma * ubq[1], gamma * ubq[2]};
        double Jb[3], t3[3];
        cross(Bq, fb, Jb);
        cross(fb, J, t3);
#pragma unroll
        for (int m = 0; m < 3; m++) Bb[m] += t3[m];
        double wb[3];
#pragma unroll
        for (int n2 = 0; n2 < 3; n2++) wb[n2] = F[0][n2] * Jb[0] + F[1][n2] * Jb[1] + F[2][n2] * Jb[2];
#pragma unroll
        for (int m = 0; m < 3; m++)
#pragma unroll
          for (int n2 = 0; n2 < 3; n2++) Fb[m][n2] += Jb[m] * w[n2];
        const double cb[3] = {wb[0] * rDq, wb[1] * rDq, wb[2] * rDq};
        rDb += wb[0] * cq[0] + wb[1] * cq[1] + wb[2] * cq[2];
        // c'_q = F'_b . G'_a - F'_a . G'_b for (a, b, q) = (1, 2, 0), (2, 0, 1), (0, 1, 2)
#pragma unroll
        for (int m = 0; m < 3; m++) {
          Fb[m][2] += cb[0] * G[1][m];
          Fb[m][1] -= cb[0] * G[2][m];
          Fb[m][0] += cb[1] * G[2][m];
          Fb[m][2] -= cb[1] * G[0][m];
          Fb[m][1] += cb[2] * G[0][m];
          Fb[m][0] -= cb[2] * G[1][m];
        }
        if constexpr (SEED) {
          double f[3];
          cross(J, Bq, f);
          Db_direct += a.seed_R2 * 0.5 * g.dV * g.inv8h3 * (f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        }
      }
      // transpose of G': Bbar(m) += sum_a Gbar'_a(m - e_a) - Gbar'_a(m + e_a)
#pragma unroll
      for (int m = 0; m < 3; m++) Bb[m] += Bbxyq[m] + (gzqm[m] - gzp[m]);
      if constexpr (SEED) {
        double zeta = 1.0;
        if (bcx == BC_LINE_TIED && (gi_t == 0 || gi_t == nx - 1)) zeta *= 0.5;
        if (bcy == BC_LINE_TIED && (gj_t == 0 || gj_t == ny - 1)) zeta *= 0.5;
        if (bcz == BC_LINE_TIED && (q == 0 || q == nz - 1)) zeta *= 0.5;
        const double kappa = a.seed_EM * zeta * g.dV * g.inv8h3;
        const double Dp = 1.0 / rDq;
#pragma unroll
        for (int m = 0; m < 3; m++) Bb[m] += kappa * Dp * Bq[m];
        Db_direct += 0.5 * kappa * (Bq[0] * Bq[0] + Bq[1] * Bq[1] + Bq[2] * Bq[2]);
      }
      // pull-back B = F' B0'' rD
      double v[3];
#pragma unroll
      for (int m = 0; m < 3; m++) v[m] = F[m][0] * b0q[0] + F[m][1] * b0q[1] + F[m][2] * b0q[2];
      rDb += Bb[0] * v[0] + Bb[1] * v[1] + Bb[2] * v[2];
#pragma unroll
      for (int m = 0; m < 3; m++)
#pragma unroll
        for (int n2 = 0; n2 < 3; n2++) Fb[m][n2] += rDq * Bb[m] * b0q[n2];
#pragma unroll
      for (int n2 = 0; n2 < 3; n2++) so_B[n2] = bbr[n2] + rDq * (F[0][n2] * Bb[0] + F[1][n2] * Bb[1] + F[2][n2] * Bb[2]);
      // det: Dbar' cof(F')
      const double Db = -rDq * rDq * rDb + Db_direct;
      double cof[3][3];
      cof[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
      cof[0][1] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
      cof[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
      cof[1][0] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
      cof[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
      cof[1][2] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
      cof[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
      cof[2][1] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
      cof[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
#pragma unroll
      for (int m = 0; m < 3; m++)
#pragma unroll
        for (int n2 = 0; n2 < 3; n2++) so_F[3 * m + n2] = Fb[m][n2] + Db * cof[m][n2];
    }
    load_point(p);  // B0bar'' at the output node of the next plane step
    store_point(q, qout);
    __syncthreads();

#pragma unroll
    for (int m = 0; m < 3; m++) {
      Fzq[m] = Fzp[m];
      ubq[m] = ubp[m];
      Bqm[m] = Bq[m];
      Bq[m] = Bp[m];
      b0q[m] = b0p[m];
      gzqm[m] = gzq[m];
      gzq[m] = gzp[m];
      Bbxyq[m] = Bbxyp[m];
    }
    rDq = rDp;
  }
}

// ybar = D^T Fbar': each column a of Fbar' is pulled back along axis a with the transposed
// difference rows (central: +1 at n+e_a, -1 at n-e_a; one-sided ends: (-3, 4, -1) and (3, -4, 1)).
// mode 0 (stage t >= 2): ybar_t = D^T Fbar' -> ybar_out, and the cotangent of k_{t-1},
//   dt (b5_{t-1} xbar + sum_{t' >= t} a_{t',t-1} ybar_{t'}) -> ubar_out;
// mode 1 (stage 1): xbar += D^T Fbar' + sum_{t=2..6} ybar_t;  mode 2 (seed): xbar = D^T Fbar'
__global__ __launch_bounds__(256) void adj_gather_kernel(AdjArgs a, int mode, int stage) {
  const Geometry& g = a.g;
  const long long N = g.N;
  const int nx = g.n[0], ny = g.n[1];
  const double dt = (mode == 0) ? *a.dt : 0.0;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(p % nx), j = (int)((p / nx) % ny), k = (int)(p / ((long long)nx * ny));
    const int id[3] = {i, j, k};
    double yb[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int ax = 0; ax < 3; ax++) {
      const int n = g.n[ax];
      const int v = id[ax];
      const long long stride = (ax == 0) ? 1 : (ax == 1 ? (long long)nx : (long long)nx * ny);
      auto col = [&](int vv, double c) {  // yb += c * Fbar'[:, ax] at the node with index vv along ax
        const long long m = p + (long long)(vv - v) * stride;
#pragma unroll
        for (int r = 0; r < 3; r++) yb[r] += c * a.Fbar[(3 * r + ax) * N + m];
      };
      if (g.bc[ax] == BC_PERIODIC) {
        col(v == 0 ? n - 1 : v - 1, 1.0);
        col(v == n - 1 ? 0 : v + 1, -1.0);
      } else {
        if (v - 1 >= 1 && v - 1 <= n - 2) col(v - 1, 1.0);
        if (v + 1 >= 1 && v + 1 <= n - 2) col(v + 1, -1.0);
        if (v == 0) col(0, -3.0);
        if (v == 1) col(0, 4.0);
        if (v == 2) col(0, -1.0);
        if (v == n - 1) col(n - 1, 3.0);
        if (v == n - 2) col(n - 1, -4.0);
        if (v == n - 3) col(n - 1, 1.0);
      }
    }
    if (mode == 0) {
      const int s = stage - 1;  // the stage whose k's cotangent is assembled
#pragma unroll
      for (int r = 0; r < 3; r++) {
        a.ybar_out[p + r * N] = yb[r];
        double v = CK::b5[s - 1] * a.xbar[p + r * N] + CK::a[stage - 1][s - 1] * yb[r];
        for (int t = stage + 1; t <= 6; t++) v += CK::a[t - 1][s - 1] * a.ybar[t][p + r * N];
        a.ubar_out[p + r * N] = dt * v;
      }
    } else if (mode == 1) {
#pragma unroll
      for (int r = 0; r < 3; r++) {
        double s = a.xbar_out[p + r * N] + yb[r];
        for (int t = 2; t <= 6; t++) s += a.ybar[t][p + r * N];
        a.xbar_out[p + r * N] = s;
      }
    } else {
#pragma unroll
      for (int r = 0; r < 3; r++) a.xbar_out[p + r * N] = yb[r];
    }
  }
}

__global__ void fill_kernel(double* __restrict__ v, long long n, double val) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    v[i] = val;
}

// the forward recompute of one recorded step runs on its own control block
__global__ void seg_step_kernel(Control* c2, const double* __restrict__ dt_record, long long n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c2->dt = dt_record[n];
    c2->status = 0;
    c2->cur = 0;
    c2->accepted = 0;
    c2->target = 1;
    c2->need_k1 = 1;
    c2->record = 0;
  }
}

template <int S, bool XYP, bool SEED>
hipError_t launch_field_t(const AdjArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((adj_field_kernel<S, XYP, SEED>), dim3(a.g.nblocks), dim3(NTHREADS), 0, st, a);
  return hipGetLastError();
}

template <bool XYP>
hipError_t launch_field_x(int s, bool seed, const AdjArgs& a, hipStream_t st) {
  if (seed) return launch_field_t<1, XYP, true>(a, st);
  switch (s) {
    case 1: return launch_field_t<1, XYP, false>(a, st);
    case 2: return launch_field_t<2, XYP, false>(a, st);
    case 3: return launch_field_t<3, XYP, false>(a, st);
    case 4: return launch_field_t<4, XYP, false>(a, st);
    case 5: return launch_field_t<5, XYP, false>(a, st);
    case 6: return launch_field_t<6, XYP, false>(a, st);
    default: return hipErrorInvalidValue;
  }
}

unsigned grid_for(long long n) {
  long long b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_adj_field(int s, bool seed, const AdjArgs& a, hipStream_t st) {
  const bool xyp = (a.g.bc[0] == BC_PERIODIC && a.g.bc[1] == BC_PERIODIC);
  return xyp ? launch_field_x<true>(s, seed, a, st) : launch_field_x<false>(s, seed, a, st);
}

hipError_t launch_adj_gather(const AdjArgs& a, int mode, int stage, hipStream_t st) {
  hipLaunchKernelGGL(adj_gather_kernel, dim3(grid_for(a.g.N)), dim3(256), 0, st, a, mode, stage);
  return hipGetLastError();
}

hipError_t launch_fill(double* v, long long n, double val, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, st, v, n, val);
  return hipGetLastError();
}

hipError_t launch_seg_step(Control* c2, const double* dt_record, long long n, hipStream_t st) {
  hipLaunchKernelGGL(seg_step_kernel, dim3(1), dim3(64), 0, st, c2, dt_record, n);
  return hipGetLastError();
}

}  // namespace relax
