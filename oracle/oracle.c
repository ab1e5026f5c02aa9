/*
 * oracle.c -- plain, slow FP64 CPU oracle of the Lagrangian mimetic magneto-frictional
 * relaxation step of Candelaresi, Pontin & Hornig, "Mimetic Methods for Lagrangian
 * Relaxation of Magnetic Fields" (SIAM J. Sci. Comput.; GLEMuR).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the package smoke check and the CPU-baseline
 * leg of the benchmark may load or call this file.  It shares no code, header, table or
 * helper with the HIP library; the two only agree on the data layout and the status codes
 * written out below.
 *
 * The file is compiled twice:
 *   * as real double            -> symbols orc_*   (everything)
 *   * with -DORACLE_COMPLEX     -> symbols orcz_*  (fixed-dt trajectory in complex
 *     arithmetic, for complex-step directional derivatives: Im f(p + i e v) / e).
 *
 * Data layout: every vector field is structure-of-arrays [3][nz][ny][nx], x fastest.
 *
 * The steps follow the paper in its own order:
 *   Jacobian F = dx/dX and Delta = det F          (Sec. 2.1, eq. "B transformation")
 *   pull-back B = F B0 / Delta                    (Sec. 2.1, eq. "B transformation")
 *   loop circulation sum_r B_r . dx_r             (Sec. 2.2, eq. "current discrete")
 *   area vector sum of four triangles             (Sec. 2.2, eqs. "four surfaces",
 *                                                  "sum of triangles")
 *   3x3 solve of J . n A = circulation            (Sec. 2.2, eq. "current matrix equation")
 *   or, selected by orc_set_curl(1), the next-nearest-neighbour loops over the octilateral
 *   of the eight in-plane ring neighbours          (Sec. 2.3, eqs. "eight surfaces",
 *                                                  "sum of eight triangles")
 *   u = gamma J x B                               (Sec. 1, eq. "magneto friction")
 *   Cash-Karp RK5(4) + step-size rule             (Sec. 2.4, eq. "time stepping")
 *   line-tied / periodic boundaries               (Sec. 2.5)
 *   magnetic energy with face weights zeta        (Sec. 3.2.4, eq. "magnetic energy")
 *   xi = max |J x B| / B^2                         (Sec. 4.1)
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   R1 F by second-order central differences, second-order one-sided at line-tied ends,
 *      wrapped with the coordinate shift on periodic axes.
 *   R2 loop vertices I..IV = the four in-plane nearest neighbours +a, +b, -a, -b,
 *      (a, b, q) cyclic.
 *   R3 n A is the vector sum of the four triangle vectors; no square roots.
 *   R4 the fifth-order solution is propagated.
 *   R5 Lambda = max over nodes and components of |x5 - x4|.
 *   R6 zeta weights apply on line-tied faces only.
 *   R7 xi skips nodes with |B|^2 <= tau_B2 (caller-given absolute threshold).
 *   R8 R2 = 1/2 sum_interior Delta |J x B|^2 dV, the smooth residual.
 *   R9 the step-size rule as printed, with an optional safety factor (1 = as printed) on
 *      the new step; when Lambda == 0 the step grows by 5x.
 *   R16 convexity: a node is concave when any of its trihedra fails the sign test; trihedra
 *      reaching beyond a line-tied face are not formed.
 *   R19 octilateral (Sec. 2.3; its figure is missing): vertices 1..8 are the ring neighbours
 *      p+e_a, p+e_a+e_b, p+e_b, p-e_a+e_b, p-e_a, p-e_a-e_b, p-e_b, p+e_a-e_b (the edge
 *      points odd, the diagonal points even); dx_r = x(V_r+1) - x(V_r); dx_A..dx_D are the
 *      edges of the quadrilateral through the diagonal points, V2 -> V4 -> V6 -> V8 -> V2.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_COMPLEX
#include <complex.h>
typedef double complex real_t;
#else
typedef double real_t;
#endif

/* status codes (same values as the product library's, by interface agreement) */
#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_FOLD (-3)
#define ORC_E_DT (-4)
#define ORC_E_NAN (-5)
#define ORC_E_MEM (-7)

#define BC_LINE_TIED 0
#define BC_PERIODIC 1

typedef struct {
  int n[3];
  double h[3];
  int bc[3];
  long N;
} grid_t;

static int grid_init(grid_t *g, const int n[3], const double h[3], const int bc[3]) {
  for (int a = 0; a < 3; a++) {
    if (n[a] < 4 || !(h[a] > 0.0) || (bc[a] != BC_LINE_TIED && bc[a] != BC_PERIODIC)) return ORC_E_ARG;
    g->n[a] = n[a];
    g->h[a] = h[a];
    g->bc[a] = bc[a];
  }
  g->N = (long)n[0] * n[1] * n[2];
  return ORC_OK;
}

static long node_id(const grid_t *g, const int p[3]) {
  return ((long)p[2] * g->n[1] + p[1]) * g->n[0] + p[0];
}

/* Neighbour access (Sec. 2.5).  Node p + d.  On a periodic axis the index wraps and the
 * coordinate of that axis is shifted by the period n*h per wrap, so a ghost carries the
 * position of its image node plus L + dZ.  Returns -1 off a line-tied axis. */
static long neighbour(const grid_t *g, const int p[3], const int d[3], double shift[3]) {
  int q[3];
  for (int a = 0; a < 3; a++) {
    int v = p[a] + d[a];
    shift[a] = 0.0;
    if (g->bc[a] == BC_PERIODIC) {
      int w = 0;
      while (v < 0) { v += g->n[a]; w -= 1; }
      while (v >= g->n[a]) { v -= g->n[a]; w += 1; }
      shift[a] = (double)w * g->n[a] * g->h[a];
    } else if (v < 0 || v >= g->n[a]) {
      return -1;
    }
    q[a] = v;
  }
  return node_id(g, q);
}

/* position x(p + d), periodic shift included */
static void position(const grid_t *g, const real_t *x, const int p[3], const int d[3], real_t out[3]) {
  double s[3];
  long m = neighbour(g, p, d, s);
  for (int c = 0; c < 3; c++) out[c] = x[c * g->N + m] + s[c];
}

static int on_line_tied_face(const grid_t *g, const int p[3]) {
  for (int a = 0; a < 3; a++)
    if (g->bc[a] == BC_LINE_TIED && (p[a] == 0 || p[a] == g->n[a] - 1)) return 1;
  return 0;
}

/* zeta (Sec. 3.2.4): 1/2 per line-tied axis on which the node is an end point */
static double zeta(const grid_t *g, const int p[3]) {
  double z = 1.0;
  for (int a = 0; a < 3; a++)
    if (g->bc[a] == BC_LINE_TIED && (p[a] == 0 || p[a] == g->n[a] - 1)) z *= 0.5;
  return z;
}

/* ---------------------------------------------------------------------------------------
 * Jacobian F_ij = dx_i/dX_j (reading R1), its determinant, and the pull-back
 * B_i = (1/Delta) sum_j F_ij B0_j  (Sec. 2.1, eq. "B transformation").
 * ------------------------------------------------------------------------------------- */
static void jacobian(const grid_t *g, const real_t *x, const int p[3], real_t F[3][3]) {
  for (int a = 0; a < 3; a++) {
    int d0[3] = {0, 0, 0}, d1[3] = {0, 0, 0}, d2[3] = {0, 0, 0};
    real_t y0[3], y1[3], y2[3];
    const double inv2h = 1.0 / (2.0 * g->h[a]);
    if (g->bc[a] == BC_PERIODIC || (p[a] > 0 && p[a] < g->n[a] - 1)) {
      d1[a] = 1;
      d2[a] = -1;
      position(g, x, p, d1, y1);
      position(g, x, p, d2, y2);
      for (int c = 0; c < 3; c++) F[c][a] = (y1[c] - y2[c]) * inv2h;
    } else if (p[a] == 0) {
      d1[a] = 1;
      d2[a] = 2;
      position(g, x, p, d0, y0);
      position(g, x, p, d1, y1);
      position(g, x, p, d2, y2);
      for (int c = 0; c < 3; c++) F[c][a] = (-3.0 * y0[c] + 4.0 * y1[c] - y2[c]) * inv2h;
    } else {
      d1[a] = -1;
      d2[a] = -2;
      position(g, x, p, d0, y0);
      position(g, x, p, d1, y1);
      position(g, x, p, d2, y2);
      for (int c = 0; c < 3; c++) F[c][a] = (3.0 * y0[c] - 4.0 * y1[c] + y2[c]) * inv2h;
    }
  }
}

static real_t det3(real_t M[3][3]) {
  return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
       - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
       + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

/* B and Delta at one node */
static void field_at(const grid_t *g, const real_t *x, const real_t *B0, const int p[3], real_t Bp[3], real_t *det) {
  const long N = g->N;
  const long m = node_id(g, p);
  real_t F[3][3];
  jacobian(g, x, p, F);
  real_t D = det3(F);
  if (det) *det = D;
  for (int c = 0; c < 3; c++) {
    real_t s = 0.0;
    for (int jj = 0; jj < 3; jj++) s += F[c][jj] * B0[jj * N + m];
    Bp[c] = s / D;
  }
}

/* B and Delta at every node */
static void pull_back(const grid_t *g, const real_t *x, const real_t *B0, real_t *B, real_t *det) {
  const long N = g->N;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g->n[2]; k++)
    for (int j = 0; j < g->n[1]; j++)
      for (int i = 0; i < g->n[0]; i++) {
        int p[3] = {i, j, k};
        long m = node_id(g, p);
        real_t Bp[3];
        field_at(g, x, B0, p, Bp, &det[m]);
        for (int c = 0; c < 3; c++) B[c * N + m] = Bp[c];
      }
}

/* ---------------------------------------------------------------------------------------
 * Mimetic current at an interior node (Sec. 2.2).
 * For the plane spanned by index axes (a, b), with q the third axis, (a, b, q) cyclic:
 *   vertices I..IV = p+e_a, p+e_b, p-e_a, p-e_b             (reading R2)
 *   circulation C_q = sum_r B_r . dx_r, B_r = (B(V_r)+B(V_r+1))/2, dx_r = x(V_r+1)-x(V_r)
 *   area vector N_q = sum_r (x(V_r)-x_p) x (x(V_r+1)-x_p) / 2
 * and J solves the three equations J . N_q = C_q (Cramer's rule, one division).
 * ------------------------------------------------------------------------------------- */
static const int PLANE_AB[3][2] = {{1, 2}, {2, 0}, {0, 1}};

static void cross(const real_t a[3], const real_t b[3], real_t out[3]) {
  out[0] = a[1] * b[2] - a[2] * b[1];
  out[1] = a[2] * b[0] - a[0] * b[2];
  out[2] = a[0] * b[1] - a[1] * b[0];
}

/* current operator: 0 = nearest-neighbour loops (Sec. 2.2), 1 = next-nearest-neighbour
 * octilateral loops (Sec. 2.3) */
static int g_curl = 0;

/* B at the node p + d, read from B or (B == NULL) pulled back from B0 on the spot */
static void vertex_field(const grid_t *g, const real_t *x, const real_t *B, const real_t *B0, long m, real_t out[3]) {
  const long N = g->N;
  if (B) {
    for (int c = 0; c < 3; c++) out[c] = B[c * N + m];
  } else {
    int q[3] = {(int)(m % g->n[0]), (int)((m / g->n[0]) % g->n[1]), (int)(m / ((long)g->n[0] * g->n[1]))};
    field_at(g, x, B0, q, out, NULL);
  }
}

/* Next-nearest-neighbour mimetic current at an interior node (Sec. 2.3).  For each plane
 * (a, b), q the third axis, the loop runs over the eight ring neighbours (reading R19):
 *   circulation C_q = sum_{r=1..8} B_r . dx_r, B_r = (B(V_r) + B(V_r+1))/2
 *   area vector N_q = (dx2 x dx3 + dx4 x dx5 + dx6 x dx7 + dx8 x dx1)/2
 *                   + (dxA x dxB + dxB x dxC + dxC x dxD + dxD x dxA)/4
 * (the four triangles at the edge points and the quadrilateral through the diagonal points,
 * eq. "eight surfaces"), and J solves J . N_q = C_q as in Sec. 2.2. */
static void octilateral_current(const grid_t *g, const real_t *x, const real_t *B, const real_t *B0, const int p[3],
                                real_t J[3]) {
  const long N = g->N;
  static const int RING[8][2] = {{1, 0}, {1, 1}, {0, 1}, {-1, 1}, {-1, 0}, {-1, -1}, {0, -1}, {1, -1}};
  real_t M[3][3], C[3];
  for (int q = 0; q < 3; q++) {
    const int a = PLANE_AB[q][0], b = PLANE_AB[q][1];
    real_t V[8][3], BV[8][3];
    for (int r = 0; r < 8; r++) {
      int off[3] = {0, 0, 0};
      off[a] = RING[r][0];
      off[b] = RING[r][1];
      double s[3];
      long m = neighbour(g, p, off, s);
      for (int c = 0; c < 3; c++) V[r][c] = x[c * N + m] + s[c];
      vertex_field(g, x, B, B0, m, BV[r]);
    }
    real_t dx[8][3], circ = 0.0;
    for (int r = 0; r < 8; r++) {
      const int r1 = (r + 1) % 8;
      for (int c = 0; c < 3; c++) {
        dx[r][c] = V[r1][c] - V[r][c];
        circ += 0.5 * (BV[r][c] + BV[r1][c]) * dx[r][c];
      }
    }
    /* dx_A..dx_D: V2 -> V4 -> V6 -> V8 -> V2 (0-based vertices 1, 3, 5, 7) */
    real_t dq[4][3];
    for (int t = 0; t < 4; t++) {
      const int v0 = 2 * t + 1, v1 = (2 * t + 3) % 8;
      for (int c = 0; c < 3; c++) dq[t][c] = V[v1][c] - V[v0][c];
    }
    real_t nA[3] = {0.0, 0.0, 0.0}, tri[3];
    /* the triangles at the edge points: dx2 x dx3, dx4 x dx5, dx6 x dx7, dx8 x dx1 (1-based) */
    for (int t = 0; t < 4; t++) {
      cross(dx[2 * t + 1], dx[(2 * t + 2) % 8], tri);
      for (int c = 0; c < 3; c++) nA[c] += 0.5 * tri[c];
    }
    /* the quadrilateral through the diagonal points */
    for (int t = 0; t < 4; t++) {
      cross(dq[t], dq[(t + 1) % 4], tri);
      for (int c = 0; c < 3; c++) nA[c] += 0.25 * tri[c];
    }
    for (int c = 0; c < 3; c++) M[q][c] = nA[c];
    C[q] = circ;
  }
  real_t dM = det3(M);
  real_t inv = 1.0 / dM;
  for (int c = 0; c < 3; c++) {
    real_t Mc[3][3];
    for (int r = 0; r < 3; r++)
      for (int s = 0; s < 3; s++) Mc[r][s] = (s == c) ? C[r] : M[r][s];
    J[c] = det3(Mc) * inv;
  }
}

/* B == NULL: the vertex fields are pulled back from B0 on the spot (sampled evaluation) */
static void mimetic_current(const grid_t *g, const real_t *x, const real_t *B, const real_t *B0, const int p[3],
                            real_t J[3]) {
  if (g_curl == 1) {
    octilateral_current(g, x, B, B0, p, J);
    return;
  }
  const long N = g->N;
  real_t M[3][3], C[3];
  real_t xp[3];
  int zero[3] = {0, 0, 0};
  position(g, x, p, zero, xp);
  for (int q = 0; q < 3; q++) {
    const int a = PLANE_AB[q][0], b = PLANE_AB[q][1];
    int off[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    off[0][a] = 1;
    off[1][b] = 1;
    off[2][a] = -1;
    off[3][b] = -1;
    real_t V[4][3], BV[4][3];
    for (int r = 0; r < 4; r++) {
      double s[3];
      long m = neighbour(g, p, off[r], s);
      for (int c = 0; c < 3; c++) V[r][c] = x[c * N + m] + s[c];
      if (B) {
        for (int c = 0; c < 3; c++) BV[r][c] = B[c * N + m];
      } else {
        int q[3] = {(int)(m % g->n[0]), (int)((m / g->n[0]) % g->n[1]), (int)(m / ((long)g->n[0] * g->n[1]))};
        field_at(g, x, B0, q, BV[r], NULL);
      }
    }
    real_t circ = 0.0, nA[3] = {0.0, 0.0, 0.0};
    for (int r = 0; r < 4; r++) {
      const int r1 = (r + 1) % 4;
      real_t dx[3], e1[3], e2[3], tri[3];
      for (int c = 0; c < 3; c++) {
        real_t Br = 0.5 * (BV[r][c] + BV[r1][c]);
        dx[c] = V[r1][c] - V[r][c];
        circ += Br * dx[c];
        e1[c] = V[r][c] - xp[c];
        e2[c] = V[r1][c] - xp[c];
      }
      cross(e1, e2, tri);
      for (int c = 0; c < 3; c++) nA[c] += 0.5 * tri[c];
    }
    for (int c = 0; c < 3; c++) M[q][c] = nA[c];
    C[q] = circ;
  }
  /* Cramer's rule */
  real_t dM = det3(M);
  real_t inv = 1.0 / dM;
  for (int c = 0; c < 3; c++) {
    real_t Mc[3][3];
    for (int r = 0; r < 3; r++)
      for (int s = 0; s < 3; s++) Mc[r][s] = (s == c) ? C[r] : M[r][s];
    J[c] = det3(Mc) * inv;
  }
}

/* ---------------------------------------------------------------------------------------
 * Right-hand side u(x) = gamma J x B, zero on line-tied faces (Sec. 2.5), plus the
 * per-node quantities the diagnostics need.
 * ------------------------------------------------------------------------------------- */
typedef struct {
  real_t *B, *det, *J;
} work_t;

static int work_alloc(const grid_t *g, work_t *w) {
  w->B = (real_t *)malloc(sizeof(real_t) * 3 * g->N);
  w->det = (real_t *)malloc(sizeof(real_t) * g->N);
  w->J = (real_t *)malloc(sizeof(real_t) * 3 * g->N);
  if (!w->B || !w->det || !w->J) {
    free(w->B); free(w->det); free(w->J);
    return ORC_E_MEM;
  }
  return ORC_OK;
}

static void work_free(work_t *w) {
  free(w->B); free(w->det); free(w->J);
}

/* u on every node; J stored (zero on line-tied faces) */
static void rhs(const grid_t *g, double gamma, const real_t *x, const real_t *B0, work_t *w, real_t *u) {
  const long N = g->N;
  pull_back(g, x, B0, w->B, w->det);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g->n[2]; k++)
    for (int j = 0; j < g->n[1]; j++)
      for (int i = 0; i < g->n[0]; i++) {
        int p[3] = {i, j, k};
        long m = node_id(g, p);
        real_t J[3] = {0.0, 0.0, 0.0}, f[3] = {0.0, 0.0, 0.0};
        if (!on_line_tied_face(g, p)) {
          real_t Bm[3] = {w->B[m], w->B[N + m], w->B[2 * N + m]};
          mimetic_current(g, x, w->B, NULL, p, J);
          cross(J, Bm, f);
        }
        for (int c = 0; c < 3; c++) {
          w->J[c * N + m] = J[c];
          u[c * N + m] = gamma * f[c];
        }
      }
}

/* ---------------------------------------------------------------------------------------
 * Cash-Karp RK5(4) tableau (Sec. 2.4; Cash & Karp 1990)
 * ------------------------------------------------------------------------------------- */
static const double CK_A[6][5] = {
    {0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0},
    {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0, 0},
    {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0},
    {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0}};
static const double CK_B5[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0};
static const double CK_B4[6] = {2825.0 / 27648.0, 0.0, 18575.0 / 48384.0, 13525.0 / 55296.0,
                                277.0 / 14336.0, 1.0 / 4.0};

/* One Cash-Karp attempt from x with step dt.  k[0] must already hold u(x).
 * Writes the fifth-order x_new and, if err != NULL, err = dt sum (b5 - b4) k. */
static void ck_attempt(const grid_t *g, double gamma, const real_t *x, const real_t *B0, real_t dt,
                       real_t *k[6], real_t *ytmp, work_t *w, real_t *x_new, real_t *err) {
  const long n3 = 3 * g->N;
  for (int s = 1; s < 6; s++) {
#pragma omp parallel for schedule(static)
    for (long e = 0; e < n3; e++) {
      real_t acc = 0.0;
      for (int j = 0; j < s; j++) acc += CK_A[s][j] * k[j][e];
      ytmp[e] = x[e] + dt * acc;
    }
    rhs(g, gamma, ytmp, B0, w, k[s]);
  }
#pragma omp parallel for schedule(static)
  for (long e = 0; e < n3; e++) {
    real_t a5 = 0.0, ae = 0.0;
    for (int s = 0; s < 6; s++) {
      a5 += CK_B5[s] * k[s][e];
      ae += (CK_B5[s] - CK_B4[s]) * k[s][e];
    }
    x_new[e] = x[e] + dt * a5;
    if (err) err[e] = dt * ae;
  }
}

/* ======================================================================================= */
#ifndef ORACLE_COMPLEX
/* ======================================================================================= */

/* diagnostics: out[0]=E_M, out[1]=xi, out[2]=min Delta, out[3]=R2, out[4]=#nodes skipped
 * by the null guard.  Uses the per-node B, Delta, J already in w. */
static void diagnostics_from_work(const grid_t *g, const work_t *w, double tau_B2, double out[5]) {
  const long N = g->N;
  const double dV = g->h[0] * g->h[1] * g->h[2];
  const int nz = g->n[2];
  double *pe = (double *)calloc(nz, sizeof(double));
  double *pr = (double *)calloc(nz, sizeof(double));
  double *px = (double *)calloc(nz, sizeof(double));
  double *pd = (double *)calloc(nz, sizeof(double));
  long *ps = (long *)calloc(nz, sizeof(long));
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; k++) {
    double e = 0.0, r = 0.0, xm = 0.0, dm = INFINITY;
    long sk = 0;
    for (int j = 0; j < g->n[1]; j++)
      for (int i = 0; i < g->n[0]; i++) {
        int p[3] = {i, j, k};
        long m = node_id(g, p);
        double Bm[3] = {w->B[m], w->B[N + m], w->B[2 * N + m]};
        double Jm[3] = {w->J[m], w->J[N + m], w->J[2 * N + m]};
        double B2 = Bm[0] * Bm[0] + Bm[1] * Bm[1] + Bm[2] * Bm[2];
        double D = w->det[m];
        e += zeta(g, p) * B2 * D;
        if (D < dm || isnan(D)) dm = D;
        if (!on_line_tied_face(g, p)) {
          double f[3];
          cross(Jm, Bm, f);
          double f2 = f[0] * f[0] + f[1] * f[1] + f[2] * f[2];
          r += D * f2;
          if (B2 > tau_B2) {
            double ratio = sqrt(f2) / B2;
            if (ratio > xm || isnan(ratio)) xm = ratio;
          } else {
            sk += 1;
          }
        }
      }
    pe[k] = e;
    pr[k] = r;
    px[k] = xm;
    pd[k] = dm;
    ps[k] = sk;
  }
  double E = 0.0, R = 0.0, X = 0.0, Dm = INFINITY;
  long S = 0;
  for (int k = 0; k < nz; k++) {
    E += pe[k];
    R += pr[k];
    if (px[k] > X || isnan(px[k])) X = px[k];
    if (pd[k] < Dm || isnan(pd[k])) Dm = pd[k];
    S += ps[k];
  }
  out[0] = 0.5 * E * dV;
  out[1] = X;
  out[2] = Dm;
  out[3] = 0.5 * R * dV;
  out[4] = (double)S;
  free(pe); free(pr); free(px); free(pd); free(ps);
}

/* Per-node fields at positions x: B (3N), det (N), J (3N), u (3N). Any output may be NULL. */
int orc_fields(const int n[3], const double h[3], const int bc[3], double gamma, const double *x,
               const double *B0, double *B, double *det, double *J, double *u) {
  grid_t g;
  work_t w;
  int rc = grid_init(&g, n, h, bc);
  if (rc) return rc;
  if ((rc = work_alloc(&g, &w))) return rc;
  double *uu = (double *)malloc(sizeof(double) * 3 * g.N);
  if (!uu) { work_free(&w); return ORC_E_MEM; }
  rhs(&g, gamma, x, B0, &w, uu);
  if (B) memcpy(B, w.B, sizeof(double) * 3 * g.N);
  if (det) memcpy(det, w.det, sizeof(double) * g.N);
  if (J) memcpy(J, w.J, sizeof(double) * 3 * g.N);
  if (u) memcpy(u, uu, sizeof(double) * 3 * g.N);
  free(uu);
  work_free(&w);
  return ORC_OK;
}

/* u = gamma J x B at the listed nodes only (flat node indices), for spot checks of grids
 * too large for a full sweep.  u_out: [count][3]. */
int orc_rhs_sampled(const int n[3], const double h[3], const int bc[3], double gamma, const double *x,
                    const double *B0, long count, const long *nodes, double *u_out) {
  grid_t g;
  int rc = grid_init(&g, n, h, bc);
  if (rc) return rc;
#pragma omp parallel for schedule(dynamic, 16)
  for (long s = 0; s < count; s++) {
    const long m = nodes[s];
    int p[3] = {(int)(m % g.n[0]), (int)((m / g.n[0]) % g.n[1]), (int)(m / ((long)g.n[0] * g.n[1]))};
    double f[3] = {0.0, 0.0, 0.0};
    if (!on_line_tied_face(&g, p)) {
      double J[3], Bm[3];
      field_at(&g, x, B0, p, Bm, NULL);
      mimetic_current(&g, x, NULL, B0, p, J);
      cross(J, Bm, f);
    }
    for (int c = 0; c < 3; c++) u_out[3 * s + c] = gamma * f[c];
  }
  return ORC_OK;
}

/* Convexity (Sec. 3.2.3, eqs. "dx for convexity", "convexity").  At node p, for each sign
 * triple (di, dj, dk) in {-1, 1}^3 the trihedron of the edge vectors from x(p) to the
 * neighbours p + di e_x, p + dj e_y, p + dk e_z; the node is convex (kappa = 1) when every
 * trihedron's determinant has the sign di dj dk, otherwise concave (kappa = -1).  Trihedra
 * that would need a neighbour beyond a line-tied face are not formed (reading R16).
 * kappa: N ints (may be NULL); *concave receives the number of concave nodes. */
#ifndef ORACLE_COMPLEX
int orc_convexity(const int n[3], const double h[3], const int bc[3], const double *x, int *kappa,
                  long *concave) {
  grid_t g;
  int rc = grid_init(&g, n, h, bc);
  if (rc) return rc;
  long count = 0;
#pragma omp parallel for reduction(+ : count) schedule(static)
  for (long m = 0; m < g.N; m++) {
    const int p[3] = {(int)(m % g.n[0]), (int)((m / g.n[0]) % g.n[1]), (int)(m / ((long)g.n[0] * g.n[1]))};
    const int zero[3] = {0, 0, 0};
    double xc[3];
    position(&g, x, p, zero, xc);
    int convex = 1;
    for (int di = -1; di <= 1; di += 2)
      for (int dj = -1; dj <= 1; dj += 2)
        for (int dk = -1; dk <= 1; dk += 2) {
          const int d[3][3] = {{di, 0, 0}, {0, dj, 0}, {0, 0, dk}};
          double e[3][3];
          int ok = 1;
          for (int v = 0; v < 3; v++) {
            double s3[3];
            if (neighbour(&g, p, d[v], s3) < 0) { ok = 0; break; }
            double xn[3];
            position(&g, x, p, d[v], xn);
            for (int c = 0; c < 3; c++) e[v][c] = xn[c] - xc[c];
          }
          if (!ok) continue;
          const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                             e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                             e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
          const double sgn = (det > 0.0) ? 1.0 : (det < 0.0 ? -1.0 : 0.0);
          if (sgn != (double)(di * dj * dk)) convex = 0;
        }
    if (kappa) kappa[m] = convex ? 1 : -1;
    count += convex ? 0 : 1;
  }
  *concave = count;
  return ORC_OK;
}
#endif

/* Diagnostics of positions x: out = {E_M, xi, min Delta, R2, skipped}. */
int orc_diagnostics(const int n[3], const double h[3], const int bc[3], double tau_B2, const double *x,
                    const double *B0, double out[5]) {
  grid_t g;
  work_t w;
  int rc = grid_init(&g, n, h, bc);
  if (rc) return rc;
  if ((rc = work_alloc(&g, &w))) return rc;
  double *u = (double *)malloc(sizeof(double) * 3 * g.N);
  if (!u) { work_free(&w); return ORC_E_MEM; }
  rhs(&g, 1.0, x, B0, &w, u);
  diagnostics_from_work(&g, &w, tau_B2, out);
  free(u);
  work_free(&w);
  return ORC_OK;
}

/* One Cash-Karp attempt with fixed dt: x_new and Lambda = max |err|. k_out (6 x 3N) optional. */
int orc_ck_attempt(const int n[3], const double h[3], const int bc[3], double gamma, const double *x,
                   const double *B0, double dt, double *x_new, double *Lambda, double *k_out) {
  grid_t g;
  work_t w;
  int rc = grid_init(&g, n, h, bc);
  if (rc) return rc;
  if ((rc = work_alloc(&g, &w))) return rc;
  const long n3 = 3 * g.N;
  double *buf = (double *)malloc(sizeof(double) * n3 * 8);
  if (!buf) { work_free(&w); return ORC_E_MEM; }
  double *k[6];
  for (int s = 0; s < 6; s++) k[s] = buf + s * n3;
  double *ytmp = buf + 6 * n3, *err = buf + 7 * n3;
  rhs(&g, gamma, x, B0, &w, k[0]);
  ck_attempt(&g, gamma, x, B0, dt, k, ytmp, &w, x_new, err);
  double L = 0.0;
  for (long e = 0; e < n3; e++) {
    double a = fabs(err[e]);
    if (a > L || isnan(a)) L = a;
  }
  if (Lambda) *Lambda = L;
  if (k_out) memcpy(k_out, buf, sizeof(double) * 6 * n3);
  free(buf);
  work_free(&w);
  return ORC_OK;
}

/* OpenMP threads the sweeps use */
/* current operator of the later calls: 0 nearest-neighbour loops (Sec. 2.2), 1 the
 * next-nearest-neighbour octilateral (Sec. 2.3) */
int orc_set_curl(int kind) {
  if (kind != 0 && kind != 1) return ORC_E_ARG;
  g_curl = kind;
  return ORC_OK;
}

int orc_threads(void) { return omp_get_max_threads(); }

/* Set the OpenMP threads of later sweeps (timing of the oracle on a given core count). */
void orc_set_threads(int n) {
  if (n >= 1) omp_set_num_threads(n);
}

/* The Cash-Karp coefficients as stored: A (6x6, row s = stage), b5, b4. */
void orc_tableau(double A[36], double b5[6], double b4[6]) {
  for (int s = 0; s < 6; s++) {
    for (int j = 0; j < 6; j++) A[6 * s + j] = (j < 5) ? CK_A[s][j] : 0.0;
    b5[s] = CK_B5[s];
    b4[s] = CK_B4[s];
  }
}

/* Step-size rule (Sec. 2.4, eq. "time stepping"):
 *   dt' = safety dt |Lambda0 / Lambda|^{0.2};
 *   Lambda > Lambda0        -> reject, redo with dt'
 *   Lambda < Lambda0 / 2    -> accept, continue with dt'
 *   otherwise               -> accept, keep dt
 * Lambda == 0 grows the step by 5x (reading R9).  safety = 1 is the rule as the paper prints
 * it; a factor below 1 (as in the Numerical Recipes stepper the paper cites for Lambda) makes
 * repeated rejects shrink dt geometrically where Lambda barely depends on dt.
 * Returns 1 for accept, 0 for reject; *dt_next receives the next dt. */
int orc_controller(double dt, double Lambda, double tol, double safety, double *dt_next) {
  double dtp = (Lambda > 0.0) ? safety * dt * pow(fabs(tol / Lambda), 0.2) : 5.0 * dt;
  if (Lambda > tol) {
    *dt_next = dtp;
    return 0;
  }
  *dt_next = (Lambda < 0.5 * tol) ? dtp : dt;
  return 1;
}

/*
 * K accepted steps.  x (3N) is advanced in place.  *t and *dt are read and written.
 * mode 1 = adaptive (controller above), 0 = fixed dt, 2 = replay (dt of step s from
 * dts_in[s]).  diag (K x 8, may be NULL) receives per step, evaluated at the state the
 * step starts from: {t, dt used, E_M, xi, R2, Lambda, min Delta, rejects}.
 * Returns a status; *done receives the number of steps completed.
 */
int orc_run(const int n[3], const double h[3], const int bc[3], double gamma, double tau_B2, int mode,
            double tol, double safety, double dt_min, int K, double *x, const double *B0, double *t, double *dt,
            const double *dts_in, double *diag, int *done) {
  grid_t g;
  work_t w;
  int rc = grid_init(&g, n, h, bc);
  if (done) *done = 0;
  if (rc) return rc;
  if (K < 0 || !(*dt > 0.0) || (mode == 2 && !dts_in)) return ORC_E_ARG;
  if ((rc = work_alloc(&g, &w))) return rc;
  const long n3 = 3 * g.N;
  double *buf = (double *)malloc(sizeof(double) * n3 * 9);
  if (!buf) { work_free(&w); return ORC_E_MEM; }
  double *k[6];
  for (int s = 0; s < 6; s++) k[s] = buf + s * n3;
  double *ytmp = buf + 6 * n3, *err = buf + 7 * n3, *xn = buf + 8 * n3;
  rc = ORC_OK;
  for (int step = 0; step < K; step++) {
    double d[5];
    rhs(&g, gamma, x, B0, &w, k[0]);
    diagnostics_from_work(&g, &w, tau_B2, d);
    if (!(d[2] > 0.0)) { rc = isnan(d[2]) ? ORC_E_NAN : ORC_E_FOLD; break; }
    if (!isfinite(d[0]) || !isfinite(d[3])) { rc = ORC_E_NAN; break; }
    if (mode == 2) *dt = dts_in[step];
    int rejects = 0;
    double Lam = 0.0, dt_used = *dt, dt_next = *dt;
    for (;;) {
      dt_used = *dt;
      ck_attempt(&g, gamma, x, B0, dt_used, k, ytmp, &w, xn, err);
      Lam = 0.0;
      for (long e = 0; e < n3; e++) {
        double a = fabs(err[e]);
        if (a > Lam || isnan(a)) Lam = a;
      }
      if (isnan(Lam) || isinf(Lam)) { rc = ORC_E_NAN; break; }
      if (mode != 1) { dt_next = dt_used; break; }
      if (orc_controller(dt_used, Lam, tol, safety, &dt_next)) break;
      rejects += 1;
      if (dt_next < dt_min) { rc = ORC_E_DT; break; }
      *dt = dt_next;
    }
    if (rc) break;
    if (diag) {
      double *e = diag + 8 * step;
      e[0] = *t; e[1] = dt_used; e[2] = d[0]; e[3] = d[1];
      e[4] = d[3]; e[5] = Lam; e[6] = d[2]; e[7] = (double)rejects;
    }
    memcpy(x, xn, sizeof(double) * n3);
    *t += dt_used;
    *dt = dt_next;
    if (done) *done = step + 1;
  }
  free(buf);
  work_free(&w);
  return rc;
}

/* ======================================================================================= */
#else /* ORACLE_COMPLEX */
/* ======================================================================================= */

/* E_M and R2 of positions x in complex arithmetic (no max / abs on this path). */
static void energy_c(const grid_t *g, const work_t *w, real_t *E, real_t *R) {
  const long N = g->N;
  const double dV = g->h[0] * g->h[1] * g->h[2];
  real_t e = 0.0, r = 0.0;
  for (int k = 0; k < g->n[2]; k++)
    for (int j = 0; j < g->n[1]; j++)
      for (int i = 0; i < g->n[0]; i++) {
        int p[3] = {i, j, k};
        long m = node_id(g, p);
        real_t Bm[3] = {w->B[m], w->B[N + m], w->B[2 * N + m]};
        real_t Jm[3] = {w->J[m], w->J[N + m], w->J[2 * N + m]};
        real_t B2 = Bm[0] * Bm[0] + Bm[1] * Bm[1] + Bm[2] * Bm[2];
        e += zeta(g, p) * B2 * w->det[m];
        if (!on_line_tied_face(g, p)) {
          real_t f[3];
          cross(Jm, Bm, f);
          r += w->det[m] * (f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        }
      }
  *E = 0.5 * e * dV;
  *R = 0.5 * r * dV;
}

/* K fixed-dt Cash-Karp steps (dt of step s = dts[s]) in complex arithmetic from (x, B0);
 * x is advanced in place; returns E_M and R2 of the final state. */
int orcz_run_fixed(const int n[3], const double h[3], const int bc[3], double gamma, int K,
                   const double *dts, real_t *x, const real_t *B0, real_t *E_out, real_t *R2_out) {
  grid_t g;
  work_t w;
  int rc = grid_init(&g, n, h, bc);
  if (rc) return rc;
  if ((rc = work_alloc(&g, &w))) return rc;
  const long n3 = 3 * g.N;
  real_t *buf = (real_t *)malloc(sizeof(real_t) * n3 * 8);
  if (!buf) { work_free(&w); return ORC_E_MEM; }
  real_t *k[6];
  for (int s = 0; s < 6; s++) k[s] = buf + s * n3;
  real_t *ytmp = buf + 6 * n3, *xn = buf + 7 * n3;
  for (int step = 0; step < K; step++) {
    rhs(&g, gamma, x, B0, &w, k[0]);
    ck_attempt(&g, gamma, x, B0, dts[step], k, ytmp, &w, xn, NULL);
    memcpy(x, xn, sizeof(real_t) * n3);
  }
  real_t *u = k[0];
  rhs(&g, gamma, x, B0, &w, u);
  energy_c(&g, &w, E_out, R2_out);
  free(buf);
  work_free(&w);
  return ORC_OK;
}

#endif
