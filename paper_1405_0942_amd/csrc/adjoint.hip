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
// Note Gbar'(n) needs only F', rD, B and ubar at n, so Bbar(m) needs the stage input on a
// 2-node halo of m, the same footprint as the forward sweep.  adj_field_kernel forms Fbar'
// (9 values per node) and accumulates B0bar''; adj_gather_kernel applies D^T.
//
// Seeds (seed_kernel mode of adj_field_kernel): E_M = 1/2 sum zeta |B|^2 det F dV adds
// kappa D' B to Bbar and 1/2 kappa |B|^2 to Dbar' (kappa = zeta dV / (8 hx hy hz));
// R2 = 1/2 sum_interior det F |f|^2 dV enters through ubar = det F dV f / gamma (read from a
// buffer) plus 1/2 |f|^2 dV / (8 hx hy hz) on Dbar'.
#include "relax_device.h"

namespace relax {
namespace {

__device__ __forceinline__ int floordiv(int a, int n) { return a >= 0 ? a / n : -((-a + n - 1) / n); }
__device__ __forceinline__ int mod3(int p) { return ((p % 3) + 3) % 3; }

struct AxisIdx {
  int i, w;
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

__device__ __forceinline__ int logical_block(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int xcd = bid & 7, j = bid >> 3;
  return xcd * q + (xcd < r ? xcd : r) + j;
}

__device__ __forceinline__ double det3(const double F[3][3]) {
  return F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
         F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
}

__device__ __forceinline__ void cross(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

template <int S, bool XYP, bool SEED>
__global__ __launch_bounds__(NTHREADS) void adj_field_kernel(AdjArgs a) {
  constexpr int NK = (S > 1) ? S - 1 : 1;
  constexpr int NP2 = (RY2 * RX2 + NTHREADS - 1) / NTHREADS;
  constexpr int NP1 = (RY1 * RX1 + NTHREADS - 1) / NTHREADS;

  const Geometry& g = a.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const long long N = g.N;
  const long long nxy = (long long)nx * ny;
  const int bcx = XYP ? BC_PERIODIC : g.bc[0];
  const int bcy = XYP ? BC_PERIODIC : g.bc[1];
  const int bcz = g.bc[2];
  const double gamma = a.gamma;

  // stage input y_S = x + dt sum_{j<S} a_Sj k_j; cotangent ubar = dt (b5_S xbar' + sum_{t>S} a_tS ybar_t)
  const double dt = SEED ? 0.0 : *a.dt;
  double cka[NK];
#pragma unroll
  for (int j = 0; j < NK; j++) cka[j] = (S > 1) ? dt * CK::a[S - 1][j] : 0.0;
  double cub[7];
#pragma unroll
  for (int t = 0; t < 7; t++) cub[t] = (t > S && t <= 6) ? dt * CK::a[t > 0 ? t - 1 : 0][S < 6 ? S - 1 : 0] : 0.0;
  const double cux = dt * CK::b5[S - 1];

  const int lb = logical_block(blockIdx.x, g.nblocks);
  const int tile_x = lb % g.tiles[0];
  const int tile_y = (lb / g.tiles[0]) % g.tiles[1];
  const int chunk = lb / (g.tiles[0] * g.tiles[1]);
  const int i0 = tile_x * TX, j0 = tile_y * TY;
  const int z0 = chunk * g.tz;
  const int z1 = min(z0 + g.tz, nz);
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;

  __shared__ double ys[3][3][RY2 * RX2];
  __shared__ double bs[3][3][RY1 * RX1];
  __shared__ double gxy[2][6][RY1 * RX1];  // Gbar'_x (0..2) and Gbar'_y (3..5), planes q and p

  // index tables (as in the forward sweep)
  int w2xy[NP2], w2w[NP2];
#pragma unroll
  for (int r = 0; r < NP2; r++) {
    const int e = tid + r * NTHREADS;
    const int row = e / RX2, col = e - row * RX2;
    const AxisIdx rx = resolve(i0 + col - 2, nx, bcx), ry = resolve(j0 + row - 2, ny, bcy);
    w2xy[r] = (e < RY2 * RX2 && rx.ok && ry.ok) ? ry.i * nx + rx.i : -1;
    w2w[r] = (ry.w << 16) + (rx.w & 0xffff);
  }
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

  auto load_plane = [&](int pz) {
    const AxisIdx rz = resolve(pz, nz, bcz);
    const long long zo = rz.i * nxy;
    const int slot = mod3(pz);
#pragma unroll
    for (int r = 0; r < NP2; r++) {
      const int e = tid + r * NTHREADS;
      if (e < RY2 * RX2) {
        double v[3] = {0.0, 0.0, 0.0};
        if (w2xy[r] >= 0) {
          const long long idx = zo + w2xy[r];
#pragma unroll
          for (int m = 0; m < 3; m++) {
            double y = a.x[idx + m * N];
            if constexpr (S > 1) {
#pragma unroll
              for (int j = 0; j < S - 1; j++) y = fma(cka[j], a.k[j][idx + m * N], y);
            }
            v[m] = y;
          }
          v[0] += (double)(short)(w2w[r] & 0xffff) * g.period[0];
          v[1] += (double)(w2w[r] >> 16) * g.period[1];
          v[2] += rz.w * g.period[2];
        }
#pragma unroll
        for (int m = 0; m < 3; m++) ys[slot][m][e] = v[m];
      }
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

  // cotangent ubar at node index idx (zero on line-tied faces)
  auto ubar_at = [&](long long idx, double ub[3]) {
#pragma unroll
    for (int m = 0; m < 3; m++) {
      double v;
      if constexpr (SEED) {
        v = a.useed ? a.useed[idx + m * N] : 0.0;
      } else {
        v = cux * a.xbar[idx + m * N];
#pragma unroll
        for (int t = S + 1; t <= 6; t++) v = fma(cub[t], a.ybar[t][idx + m * N], v);
      }
      ub[m] = v;
    }
  };

  const bool perz = (bcz == BC_PERIODIC);
  const int pb0 = perz ? z0 - 1 : max(z0 - 1, 0);
  const int pb1 = perz ? z1 : min(z1, nz - 1);
  auto need_hi = [&](int p) { return perz ? p + 1 : (p == 0 ? 2 : (p == nz - 1 ? p : p + 1)); };
  auto need_lo = [&](int p) { return perz ? p - 1 : (p == 0 ? 0 : (p == nz - 1 ? p - 2 : p - 1)); };
  auto face_at = [&](int gi, int gj, int p) {
    return (bcx == BC_LINE_TIED && (gi == 0 || gi == nx - 1)) || (bcy == BC_LINE_TIED && (gj == 0 || gj == ny - 1)) ||
           (bcz == BC_LINE_TIED && (p == 0 || p == nz - 1));
  };

  const int gi_t = i0 + tx, gj_t = j0 + ty;
  const bool tile_ok = (gi_t < nx) && (gj_t < ny);

  double Fprev[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, Fcur[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double rDprev = 0.0, rDcur = 0.0;
  double ubprev[3] = {0, 0, 0}, ubcur[3] = {0, 0, 0};
  double gzm[3] = {0, 0, 0}, gzq[3] = {0, 0, 0}, gzp[3] = {0, 0, 0};  // Gbar'_z at the tile point, planes q-1, q, q+1

  int loaded_hi = need_lo(pb0) - 1;
  for (int p = pb0; p <= pb1 + 1; p++) {
    if (p <= pb1) {
      if (loaded_hi < need_lo(p) - 1) loaded_hi = need_lo(p) - 1;
      while (loaded_hi < need_hi(p)) load_plane(++loaded_hi);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 3; m++) gzp[m] = 0.0;
    if (p <= pb1) {
      const int sp = mod3(p), gb = p & 1;
      const long long zo = resolve(p, nz, bcz).i * nxy;
#pragma unroll
      for (int r = 0; r < NP1; r++) {
        if (f1r[r] >= 0) {
          const int r1 = f1r[r], c1 = f1c[r];
          const int gi = i0 + c1 - 1, gj = j0 + r1 - 1;
          double B[3] = {0, 0, 0}, Gx[3] = {0, 0, 0}, Gy[3] = {0, 0, 0}, Gz[3] = {0, 0, 0}, ub[3] = {0, 0, 0};
          if (f1xy[r] >= 0) {
            const long long idx = zo + f1xy[r];
            double F[3][3];
            jacobian(r1 + 1, c1 + 1, p, gi, gj, F);
            const double rD = 1.0 / det3(F);
            const double q0 = a.B0[idx], q1 = a.B0[idx + N], q2 = a.B0[idx + 2 * N];
#pragma unroll
            for (int m = 0; m < 3; m++) B[m] = (F[m][0] * q0 + F[m][1] * q1 + F[m][2] * q2) * rD;
            if (!face_at(gi, gj, p)) {
              ubar_at(idx, ub);
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
#pragma unroll
                for (int n2 = 0; n2 < 3; n2++) Fcur[m][n2] = F[m][n2];
                ubcur[m] = ub[m];
                gzp[m] = Gz[m];
              }
              rDcur = rD;
            }
          }
          const int o = r1 * RX1 + c1;
#pragma unroll
          for (int m = 0; m < 3; m++) {
            bs[sp][m][o] = B[m];
            gxy[gb][m][o] = Gx[m];
            gxy[gb][3 + m][o] = Gy[m];
          }
        }
      }
    }
    __syncthreads();

    const int q = p - 1;
    if (q >= z0 && q < z1 && tile_ok) {
      const AxisIdx rzq = resolve(q, nz, bcz);
      const long long idx = rzq.i * nxy + (long long)gj_t * nx + gi_t;
      const int o = (ty + 1) * RX1 + (tx + 1);
      const int sq = mod3(q), gb = q & 1;
      const bool interior = !face_at(gi_t, gj_t, q);
      const double Bm[3] = {bs[sq][0][o], bs[sq][1][o], bs[sq][2][o]};
      double Bb[3] = {0, 0, 0};
      double Fb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      double rDb = 0.0, Db_direct = 0.0;
      if (interior) {
        const int sm = mod3(q - 1), spl = mod3(q + 1);
        double G[3][3];  // G[a][m]
#pragma unroll
        for (int m = 0; m < 3; m++) {
          G[0][m] = bs[sq][m][o + 1] - bs[sq][m][o - 1];
          G[1][m] = bs[sq][m][o + RX1] - bs[sq][m][o - RX1];
          G[2][m] = bs[spl][m][o] - bs[sm][m][o];
        }
        const double(&F)[3][3] = Fprev;
        double cq[3];
        cq[0] = F[0][2] * G[1][0] + F[1][2] * G[1][1] + F[2][2] * G[1][2] -
                (F[0][1] * G[2][0] + F[1][1] * G[2][1] + F[2][1] * G[2][2]);
        cq[1] = F[0][0] * G[2][0] + F[1][0] * G[2][1] + F[2][0] * G[2][2] -
                (F[0][2] * G[0][0] + F[1][2] * G[0][1] + F[2][2] * G[0][2]);
        cq[2] = F[0][1] * G[0][0] + F[1][1] * G[0][1] + F[2][1] * G[0][2] -
                (F[0][0] * G[1][0] + F[1][0] * G[1][1] + F[2][0] * G[1][2]);
        const double w[3] = {cq[0] * rDprev, cq[1] * rDprev, cq[2] * rDprev};
        double J[3];
#pragma unroll
        for (int m = 0; m < 3; m++) J[m] = F[m][0] * w[0] + F[m][1] * w[1] + F[m][2] * w[2];
        const double fb[3] = {gamma * ubprev[0], gamma * ubprev[1], gamma * ubprev[2]};
        double Jb[3], t3[3];
        cross(Bm, fb, Jb);
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
        const double cb[3] = {wb[0] * rDprev, wb[1] * rDprev, wb[2] * rDprev};
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
          cross(J, Bm, f);
          Db_direct += a.seed_R2 * 0.5 * g.dV * g.inv8h3 * (f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        }
      }
      // transpose of G': Bbar(m) += sum_a Gbar'_a(m - e_a) - Gbar'_a(m + e_a)
#pragma unroll
      for (int m = 0; m < 3; m++) {
        Bb[m] += gxy[gb][m][o - 1] - gxy[gb][m][o + 1];
        Bb[m] += gxy[gb][3 + m][o - RX1] - gxy[gb][3 + m][o + RX1];
        Bb[m] += gzm[m] - gzp[m];
      }
      const double(&F)[3][3] = Fprev;
      if constexpr (SEED) {
        double zeta = 1.0;
        if (bcx == BC_LINE_TIED && (gi_t == 0 || gi_t == nx - 1)) zeta *= 0.5;
        if (bcy == BC_LINE_TIED && (gj_t == 0 || gj_t == ny - 1)) zeta *= 0.5;
        if (bcz == BC_LINE_TIED && (q == 0 || q == nz - 1)) zeta *= 0.5;
        const double kappa = a.seed_EM * zeta * g.dV * g.inv8h3;
        const double Dp = 1.0 / rDprev;
#pragma unroll
        for (int m = 0; m < 3; m++) Bb[m] += kappa * Dp * Bm[m];
        Db_direct += 0.5 * kappa * (Bm[0] * Bm[0] + Bm[1] * Bm[1] + Bm[2] * Bm[2]);
      }
      // pull-back B = F' B0'' rD
      const double q0 = a.B0[idx], q1 = a.B0[idx + N], q2 = a.B0[idx + 2 * N];
      const double b0v[3] = {q0, q1, q2};
      double v[3];
#pragma unroll
      for (int m = 0; m < 3; m++) v[m] = F[m][0] * q0 + F[m][1] * q1 + F[m][2] * q2;
      rDb += Bb[0] * v[0] + Bb[1] * v[1] + Bb[2] * v[2];
#pragma unroll
      for (int m = 0; m < 3; m++)
#pragma unroll
        for (int n2 = 0; n2 < 3; n2++) Fb[m][n2] += rDprev * Bb[m] * b0v[n2];
#pragma unroll
      for (int n2 = 0; n2 < 3; n2++)
        a.B0bar[idx + n2 * N] += rDprev * (F[0][n2] * Bb[0] + F[1][n2] * Bb[1] + F[2][n2] * Bb[2]);
      // det: Dbar' cof(F')
      const double Db = -rDprev * rDprev * rDb + Db_direct;
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
        for (int n2 = 0; n2 < 3; n2++) a.Fbar[(3 * m + n2) * N + idx] = Fb[m][n2] + Db * cof[m][n2];
    }
    // rotate the carried tile-point values
#pragma unroll
    for (int m = 0; m < 3; m++) {
#pragma unroll
      for (int n2 = 0; n2 < 3; n2++) Fprev[m][n2] = Fcur[m][n2];
      ubprev[m] = ubcur[m];
      gzm[m] = gzq[m];
      gzq[m] = gzp[m];
    }
    rDprev = rDcur;
  }
}

// ybar(p) = D^T Fbar': each column a of Fbar' is pulled back along axis a with the transposed
// difference rows (central: +1 at n+e_a, -1 at n-e_a; one-sided ends: (-3, 4, -1) and (3, -4, 1)).
// mode 0: ybar_out = D^T Fbar';  mode 1: xbar += D^T Fbar' + sum_{t=2..6} ybar_t;  mode 2: xbar = D^T Fbar'
__global__ __launch_bounds__(256) void adj_gather_kernel(AdjArgs a, int mode) {
  const Geometry& g = a.g;
  const long long N = g.N;
  const int nx = g.n[0], ny = g.n[1];
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
#pragma unroll
      for (int r = 0; r < 3; r++) a.ybar_out[p + r * N] = yb[r];
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

hipError_t launch_adj_gather(const AdjArgs& a, int mode, hipStream_t st) {
  hipLaunchKernelGGL(adj_gather_kernel, dim3(grid_for(a.g.N)), dim3(256), 0, st, a, mode);
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
