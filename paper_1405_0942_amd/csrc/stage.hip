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
// Per node the operator is two radius-1 stencils joined by pointwise maps:
//   F   = dx/dX by central differences (one-sided second order on line-tied ends,
//         wrapped with the +-period coordinate shift on periodic axes, Sec. 2.5)
//   B   = F B0 / det F                                   (eq. "B transformation")
//   G_a = central difference of B along index axis a
//   J   = F c / det F,  c_q = (F e_b) . G_a - (F e_a) . G_b   ((a, b, q) cyclic)
// The last line is the Stokes-loop current of Sec. 2.2 (eqs. "current discrete", "four
// surfaces", "current matrix equation") in closed form: on the diamond of the four
// in-plane neighbours the edge-averaged circulation is 2 h_a h_b c_q and the sum of the
// four triangle vectors is 2 h_a h_b (F e_a) x (F e_b), so the 3x3 system of the paper
// is (cof F)^T J = c, solved by J = F c / det F.
//
// Data flow: a workgroup owns a 64 x 4 (x, y) tile and marches up a z-chunk.  Each
// plane of the stage input y (tile + 2-node halo, FP64) is assembled from x_n and the
// k_j straight into an LDS ring of three planes; F, det F and B are formed on the tile
// + 1-node halo into an LDS ring of three B planes; the current, force and velocity are
// then formed on the tile one plane behind.  Every global array is read once per
// workgroup plane, coalesced along x; halo re-reads hit L2.
#include <type_traits>

#include "relax_device.h"

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

template <int S, bool MIXED>
__global__ __launch_bounds__(NTHREADS) void stage_kernel(SweepArgs a) {
  using T = typename std::conditional<MIXED, float, double>::type;
  constexpr bool STAGE1 = (S == 1);
  constexpr bool LAST = (S == 6);

  Control* ctl = a.ctl;
  const bool diag_only = (a.diag_only != 0);
  int cur;
  double dt = 0.0, gamma = 1.0, tau_B2 = 0.0;
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
  gamma = ctl->gamma;
  tau_B2 = ctl->tau_B2;

  const Geometry& g = a.g;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const long long N = g.N;
  const int bcx = g.bc[0], bcy = g.bc[1], bcz = g.bc[2];

  const int lb = logical_block(blockIdx.x, g.nblocks);
  const int tile_x = lb % g.tiles[0];
  const int tile_y = (lb / g.tiles[0]) % g.tiles[1];
  const int chunk = lb / (g.tiles[0] * g.tiles[1]);
  const int i0 = tile_x * TX, j0 = tile_y * TY;
  const int z0 = chunk * g.tz;
  const int z1 = min(z0 + g.tz, nz);

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;

  __shared__ double ys[3][3][RY2][RX2];
  __shared__ T bs[3][3][RY1][RX1];
  __shared__ double red[NTHREADS / 64][NPART];

  const double* __restrict__ xn = a.x[cur];

  // ---- stage input plane pz -> y ring --------------------------------------------------
  auto load_plane = [&](int pz) {
    const AxisIdx rz = resolve(pz, nz, bcz);
    const int slot = mod3(pz);
    const double shz = rz.w * g.period[2];
    for (int e = tid; e < RY2 * RX2; e += NTHREADS) {
      const int row = e / RX2, col = e - row * RX2;
      const AxisIdx rx = resolve(i0 + col - 2, nx, bcx);
      const AxisIdx ry = resolve(j0 + row - 2, ny, bcy);
      double v0 = 0.0, v1 = 0.0, v2 = 0.0;
      if (rx.ok && ry.ok) {
        const long long idx = ((long long)rz.i * ny + ry.i) * nx + rx.i;
        v0 = xn[idx];
        v1 = xn[idx + N];
        v2 = xn[idx + 2 * N];
        if constexpr (S > 1) {
          double c0 = 0.0, c1 = 0.0, c2 = 0.0;
#pragma unroll
          for (int j = 0; j < S - 1; j++) {
            const T* __restrict__ kj = static_cast<const T*>(a.k[j]);
            const double aj = CK::a[S - 1][j];
            c0 += aj * (double)kj[idx];
            c1 += aj * (double)kj[idx + N];
            c2 += aj * (double)kj[idx + 2 * N];
          }
          v0 += dt * c0;
          v1 += dt * c1;
          v2 += dt * c2;
        }
        v0 += rx.w * g.period[0];
        v1 += ry.w * g.period[1];
        v2 += shz;
      }
      ys[slot][0][row][col] = v0;
      ys[slot][1][row][col] = v1;
      ys[slot][2][row][col] = v2;
    }
  };

  // ---- Jacobian at a window point (r, c in stage-input window coordinates) of plane p --
  auto jacobian = [&](int r, int c, int p, int gi, int gj, double F[3][3]) {
    const int sp = mod3(p);
#pragma unroll
    for (int m = 0; m < 3; m++) {
      if (bcx == BC_PERIODIC || (gi > 0 && gi < nx - 1))
        F[m][0] = (ys[sp][m][r][c + 1] - ys[sp][m][r][c - 1]) * g.inv2h[0];
      else if (gi == 0)
        F[m][0] = (-3.0 * ys[sp][m][r][c] + 4.0 * ys[sp][m][r][c + 1] - ys[sp][m][r][c + 2]) * g.inv2h[0];
      else
        F[m][0] = (3.0 * ys[sp][m][r][c] - 4.0 * ys[sp][m][r][c - 1] + ys[sp][m][r][c - 2]) * g.inv2h[0];
      if (bcy == BC_PERIODIC || (gj > 0 && gj < ny - 1))
        F[m][1] = (ys[sp][m][r + 1][c] - ys[sp][m][r - 1][c]) * g.inv2h[1];
      else if (gj == 0)
        F[m][1] = (-3.0 * ys[sp][m][r][c] + 4.0 * ys[sp][m][r + 1][c] - ys[sp][m][r + 2][c]) * g.inv2h[1];
      else
        F[m][1] = (3.0 * ys[sp][m][r][c] - 4.0 * ys[sp][m][r - 1][c] + ys[sp][m][r - 2][c]) * g.inv2h[1];
      if (bcz == BC_PERIODIC || (p > 0 && p < nz - 1))
        F[m][2] = (ys[mod3(p + 1)][m][r][c] - ys[mod3(p - 1)][m][r][c]) * g.inv2h[2];
      else if (p == 0)
        F[m][2] = (-3.0 * ys[mod3(0)][m][r][c] + 4.0 * ys[mod3(1)][m][r][c] - ys[mod3(2)][m][r][c]) * g.inv2h[2];
      else
        F[m][2] = (3.0 * ys[mod3(p)][m][r][c] - 4.0 * ys[mod3(p - 1)][m][r][c] + ys[mod3(p - 2)][m][r][c]) *
                  g.inv2h[2];
    }
  };

  // B planes this chunk needs, and the y planes behind them
  const bool perz = (bcz == BC_PERIODIC);
  const int pb0 = perz ? z0 - 1 : max(z0 - 1, 0);
  const int pb1 = perz ? z1 : min(z1, nz - 1);
  auto need_hi = [&](int p) { return perz ? p + 1 : (p == 0 ? 2 : (p == nz - 1 ? p : p + 1)); };
  auto need_lo = [&](int p) { return perz ? p - 1 : (p == 0 ? 0 : (p == nz - 1 ? p - 2 : p - 1)); };

  // tile point owned by this thread
  const int gi_t = i0 + tx, gj_t = j0 + ty;
  const bool tile_ok = (gi_t < nx) && (gj_t < ny);

  double Fprev[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double Fcur[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double invD_prev = 0.0, invD_cur = 0.0, D_prev = 0.0, D_cur = 0.0;

  // reductions
  double acc_E = 0.0, acc_R2 = 0.0, acc_xi = 0.0, acc_min = INFINITY, acc_null = 0.0, acc_lam = 0.0;

  int loaded_hi = need_lo(pb0) - 1;
  for (int p = pb0; p <= pb1 + 1; p++) {
    // 1. stage-input planes up to need_hi(p)
    if (p <= pb1) {
      const int hi = need_hi(p);
      if (loaded_hi < need_lo(p) - 1) loaded_hi = need_lo(p) - 1;
      while (loaded_hi < hi) {
        loaded_hi++;
        load_plane(loaded_hi);
      }
    }
    __syncthreads();
    // 2. F, det F, B on the tile + 1-node halo of plane p
    if (p <= pb1) {
      const int sp = mod3(p);
      const AxisIdx rz = resolve(p, nz, bcz);
      for (int e = tid; e < RY1 * RX1; e += NTHREADS) {
        int r1, c1;
        if (e < NTHREADS) {  // tile points first, so that thread tid owns its tile point
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
        const int gi = i0 + c1 - 1, gj = j0 + r1 - 1;
        const AxisIdx rx = resolve(gi, nx, bcx), ry = resolve(gj, ny, bcy);
        T B[3] = {T(0), T(0), T(0)};
        if (rx.ok && ry.ok) {
          double F[3][3];
          jacobian(r1 + 1, c1 + 1, p, gi, gj, F);
          const double D = det3(F);
          const double invD = 1.0 / D;
          const long long idx = ((long long)rz.i * ny + ry.i) * nx + rx.i;
          const T* __restrict__ b0 = static_cast<const T*>(a.B0);
          const T q0 = b0[idx], q1 = b0[idx + N], q2 = b0[idx + 2 * N];
          if constexpr (MIXED) {
            const float fi = (float)invD;
#pragma unroll
            for (int m = 0; m < 3; m++)
              B[m] = ((float)F[m][0] * q0 + (float)F[m][1] * q1 + (float)F[m][2] * q2) * fi;
          } else {
#pragma unroll
            for (int m = 0; m < 3; m++) B[m] = (F[m][0] * q0 + F[m][1] * q1 + F[m][2] * q2) * invD;
          }
          if (e < NTHREADS) {
#pragma unroll
            for (int m = 0; m < 3; m++)
#pragma unroll
              for (int n2 = 0; n2 < 3; n2++) Fcur[m][n2] = F[m][n2];
            invD_cur = invD;
            D_cur = D;
            if (STAGE1 && p >= z0 && p < z1 && gi < nx && gj < ny) {
              // energy in FP64 from the FP64 Jacobian and B0, weights zeta on line-tied faces
              double zeta = 1.0;
              if (bcx == BC_LINE_TIED && (gi == 0 || gi == nx - 1)) zeta *= 0.5;
              if (bcy == BC_LINE_TIED && (gj == 0 || gj == ny - 1)) zeta *= 0.5;
              if (bcz == BC_LINE_TIED && (p == 0 || p == nz - 1)) zeta *= 0.5;
              double Bd[3];
#pragma unroll
              for (int m = 0; m < 3; m++)
                Bd[m] = (F[m][0] * (double)q0 + F[m][1] * (double)q1 + F[m][2] * (double)q2) * invD;
              acc_E += zeta * (Bd[0] * Bd[0] + Bd[1] * Bd[1] + Bd[2] * Bd[2]) * D;
              acc_min = (D < acc_min || D != D) ? D : acc_min;
              if (record_ck) {
                double* ck = a.ckpt + ck_slot * 3 * N;
                ck[idx] = xn[idx];
                ck[idx + N] = xn[idx + N];
                ck[idx + 2 * N] = xn[idx + 2 * N];
              }
            }
          }
        }
        bs[sp][0][r1][c1] = B[0];
        bs[sp][1][r1][c1] = B[1];
        bs[sp][2][r1][c1] = B[2];
      }
    }
    __syncthreads();
    // 3. current, force and velocity on the tile of plane q = p - 1
    const int q = p - 1;
    if (q >= z0 && q < z1 && tile_ok) {
      const AxisIdx rz = resolve(q, nz, bcz);
      const long long idx = ((long long)rz.i * ny + gj_t) * nx + gi_t;
      const bool face = (bcx == BC_LINE_TIED && (gi_t == 0 || gi_t == nx - 1)) ||
                        (bcy == BC_LINE_TIED && (gj_t == 0 || gj_t == ny - 1)) ||
                        (bcz == BC_LINE_TIED && (q == 0 || q == nz - 1));
      T u[3] = {T(0), T(0), T(0)};
      if (!face) {
        const int r = ty + 1, c = tx + 1;
        const int sq = mod3(q), sm = mod3(q - 1), spl = mod3(q + 1);
        const T ix = (T)g.inv2h[0], iy = (T)g.inv2h[1], iz = (T)g.inv2h[2];
        T G[3][3];  // G[a][m] = d B_m / d X_a
#pragma unroll
        for (int m = 0; m < 3; m++) {
          G[0][m] = (bs[sq][m][r][c + 1] - bs[sq][m][r][c - 1]) * ix;
          G[1][m] = (bs[sq][m][r + 1][c] - bs[sq][m][r - 1][c]) * iy;
          G[2][m] = (bs[spl][m][r][c] - bs[sm][m][r][c]) * iz;
        }
        T Fq[3][3];
#pragma unroll
        for (int m = 0; m < 3; m++)
#pragma unroll
          for (int n2 = 0; n2 < 3; n2++) Fq[m][n2] = (T)Fprev[m][n2];
        // c_q = (F e_b) . G_a - (F e_a) . G_b, (a, b, q) = (y, z, x), (z, x, y), (x, y, z)
        T cq[3];
        cq[0] = Fq[0][2] * G[1][0] + Fq[1][2] * G[1][1] + Fq[2][2] * G[1][2] -
                (Fq[0][1] * G[2][0] + Fq[1][1] * G[2][1] + Fq[2][1] * G[2][2]);
        cq[1] = Fq[0][0] * G[2][0] + Fq[1][0] * G[2][1] + Fq[2][0] * G[2][2] -
                (Fq[0][2] * G[0][0] + Fq[1][2] * G[0][1] + Fq[2][2] * G[0][2]);
        cq[2] = Fq[0][1] * G[0][0] + Fq[1][1] * G[0][1] + Fq[2][1] * G[0][2] -
                (Fq[0][0] * G[1][0] + Fq[1][0] * G[1][1] + Fq[2][0] * G[1][2]);
        const T iD = (T)invD_prev;
        T J[3];
#pragma unroll
        for (int m = 0; m < 3; m++) J[m] = (Fq[m][0] * cq[0] + Fq[m][1] * cq[1] + Fq[m][2] * cq[2]) * iD;
        const T Bq0 = bs[sq][0][r][c], Bq1 = bs[sq][1][r][c], Bq2 = bs[sq][2][r][c];
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
          acc_R2 += D_prev * F2;
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
          a.u_out[idx] = (double)u[0];
          a.u_out[idx + N] = (double)u[1];
          a.u_out[idx + 2 * N] = (double)u[2];
        }
      } else {
        if constexpr (!LAST) {
          T* __restrict__ ks = static_cast<T*>(a.k[S - 1]);
          ks[idx] = u[0];
          ks[idx + N] = u[1];
          ks[idx + 2 * N] = u[2];
        } else {
          // x_{n+1} = x_n + dt sum b5_s k_s;  err = dt sum (b5_s - b4_s) k_s
          double* __restrict__ xo = a.xout[1 - cur];
          const T* k1 = static_cast<const T*>(a.k[0]);
          const T* k3 = static_cast<const T*>(a.k[2]);
          const T* k4 = static_cast<const T*>(a.k[3]);
          const T* k5 = static_cast<const T*>(a.k[4]);
#pragma unroll
          for (int m = 0; m < 3; m++) {
            const long long e = idx + m * N;
            const double v1 = k1[e], v3 = k3[e], v4 = k4[e], v5 = k5[e], v6 = (double)u[m];
            const double s5 = CK::b5[0] * v1 + CK::b5[2] * v3 + CK::b5[3] * v4 + CK::b5[5] * v6;
            const double se = (CK::b5[0] - CK::b4[0]) * v1 + (CK::b5[2] - CK::b4[2]) * v3 +
                              (CK::b5[3] - CK::b4[3]) * v4 + (CK::b5[4] - CK::b4[4]) * v5 +
                              (CK::b5[5] - CK::b4[5]) * v6;
            xo[e] = xn[e] + dt * s5;
            const double err = fabs(dt * se);
            acc_lam = (err > acc_lam || err != err) ? err : acc_lam;
          }
        }
      }
    }
    // Fcur -> Fprev for the next plane
#pragma unroll
    for (int m = 0; m < 3; m++)
#pragma unroll
      for (int n2 = 0; n2 < 3; n2++) Fprev[m][n2] = Fcur[m][n2];
    invD_prev = invD_cur;
    D_prev = D_cur;
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

}  // namespace

hipError_t launch_stage(int s, bool mixed, const SweepArgs& a, hipStream_t st) {
  const dim3 grid(a.g.nblocks), block(NTHREADS);
#define RELAX_STAGE_CASE(S)                                                            \
  case S:                                                                              \
    if (mixed)                                                                         \
      hipLaunchKernelGGL((stage_kernel<S, true>), grid, block, 0, st, a);             \
    else                                                                               \
      hipLaunchKernelGGL((stage_kernel<S, false>), grid, block, 0, st, a);            \
    break;
  switch (s) {
    RELAX_STAGE_CASE(1)
    RELAX_STAGE_CASE(2)
    RELAX_STAGE_CASE(3)
    RELAX_STAGE_CASE(4)
    RELAX_STAGE_CASE(5)
    RELAX_STAGE_CASE(6)
    default:
      return hipErrorInvalidValue;
  }
#undef RELAX_STAGE_CASE
  return hipGetLastError();
}

hipError_t launch_diagnostics(const SweepArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((stage_kernel<1, false>), dim3(a.g.nblocks), dim3(NTHREADS), 0, st, a);
  return hipGetLastError();
}

}  // namespace relax
