// relax_device.h -- internal types shared by the library's translation units (kernels and
// the C-ABI glue).  Not part of the public interface (that is include/relax.h).
#pragma once

#include <hip/hip_runtime.h>

#include "relax.h"

#include <cstddef>
#include <cstdint>

namespace relax {

// ------------------------------------------------------------------------------------------
// Tiling of the fused stage sweep.  One workgroup owns a TX x TY column of nodes in (x, y)
// and marches up a z-chunk of TZ planes; one wave64 covers one x-row of the tile.
// ------------------------------------------------------------------------------------------
#ifndef RELAX_TILE_Y
#define RELAX_TILE_Y 8  // another height is built only to check that results do not depend on it
#endif
constexpr int TX = 64;
constexpr int TY = RELAX_TILE_Y;
constexpr int NTHREADS = TX * TY;  // 512 = 8 waves; one workgroup per CU (LDS: 91 KB in FP64)
constexpr int RX2 = TX + 4, RY2 = TY + 4;  // stage-input window (2-node halo)
constexpr int RX1 = TX + 2, RY1 = TY + 2;  // pulled-back field window (1-node halo)
constexpr int NPART = 8;                   // doubles per workgroup partial record
constexpr int RING_CAP = 4096;             // per-call diagnostics ring entries

enum { BC_LINE_TIED = 0, BC_PERIODIC = 1 };
enum { CURL_NN = 0, CURL_NNN = 1 };  // the values of RELAX_CURL_NN / RELAX_CURL_NNN

struct Geometry {
  int n[3];          // nodes along x, y, z
  int bc[3];         // BC_LINE_TIED / BC_PERIODIC per axis
  double h[3];       // reference spacing
  double period[3];  // n h (used on periodic axes)
  long long N;       // number of nodes
  double dV;         // hx hy hz
  double inv8h3;     // 1 / (8 hx hy hz): det F = det F' * inv8h3 for the unscaled differences F'
  double b0scale[3]; // 4 h_b h_c: B0'' = B0 * b0scale (component-wise), see stage.hip
  int tiles[3];      // tiles along x, along y, z-chunks
  int tz;            // z-chunk length
  int nblocks;       // tiles[0] * tiles[1] * tiles[2]
  int curl;          // CURL_NN: loops over the four nearest neighbours (Sec. 2.2); CURL_NNN:
                     // the octilateral over the eight ring neighbours (Sec. 2.3)
};

// Device-resident step state.  Written only by the control kernel (and by small set-up
// kernels launched by the host on the same stream).
struct Control {
  double t, dt;              // time and step to try next
  double tol, dt_min;        // Lambda_0, breakdown threshold
  double safety;             // factor on the new step of the step-size rule
  double gamma, tau_B2;      // friction coefficient, xi null-guard threshold on |B|^2
  double dV;                 // hx hy hz
  double E, xi, R2, min_det, nulls;  // diagnostics of the state x_n the current step starts from
  double lambda;             // Lambda of the last attempt
  int status;                // 0 or a (sticky) RELAX_E_* code
  int cur;                   // index of the x buffer holding x_n
  int accepted;              // accepted steps in the current relax_step chunk
  int target;                // kernels stop doing work once accepted >= target
  int need_k1;               // 1: k1 and the diagnostics of x_n are (re)computed by stage 1
  int rejects;               // rejects in the current step
  int adaptive;              // 1: step-size rule; 0: fixed dt
  int record;                // 1: store dt per step and x every `ck_every` steps
  int ck_every;              // checkpoint interval
  int record_cap;            // capacity of the dt record (steps)
  long long steps_total;     // accepted steps since init / set_state
};

// Arguments of every sweep kernel (passed by value in the kernarg segment).
struct SweepArgs {
  Geometry g;
  const double* x[2];  // position buffers (x_n is x[ctl->cur])
  double* xout[2];     // same buffers, writable (stage 6 writes x[1 - cur])
  void* k[3];          // stage vectors k_1..k_3 (double, or float in mixed mode)
  double* y3;          // stage input y_3, written by stage 2
  void* d4;            // stage-4 increment d_4 (element type of k), written by stage 3
  double* y5;          // stage input y_5, written by stage 4
  void* sum[3];        // partial sums P6 (d_6 after stage 5), X, E (element type of k; see stage.hip)
  double* yrec[2];     // forward replay of the reverse pass: y_4 and y_6 at the node
  const void* B0;      // initial field (double, or float in mixed mode)
  Control* ctl;
  double* part;        // [nblocks][NPART] reduction partials of stage 1 / diagnostics
  double* lam_part;    // [nblocks] Lambda partials of stage 6
  double* ckpt;        // checkpoint store [slots][3N] (record mode), may be null
  int ckpt_slots;
  int diag_buf;        // diagnostics sweep (launch_diagnostics) of x[diag_buf]
  double* u_out;       // diagnostics sweep only: if not null, receives u(x) [3][N] (FP64)
  double u_det_scale;  // diagnostics sweep only: if not 0, u_out holds u * det F * u_det_scale
  double* B_out;       // diagnostics sweep only: if not null, receives B(x) [3][N]
  double* J_out;       // diagnostics sweep only: if not null, receives J(x) [3][N] (0 on line-tied faces)
  double* alpha_out;   // diagnostics sweep only: if not null, receives alpha* = J.B / B^2 [N]
  int* kappa_out;      // diagnostics sweep only: if not null, receives the convexity +1 / -1 [N]
  double b0_mul[3];    // diagnostics sweep only: factors on B0 as loaded (1 for the prescaled
                       // copy B0''; 4 h_b h_c for a caller's unscaled B0)
};

// Arguments of the reverse-mode sweeps (adjoint.hip).  FP64 throughout.
struct AdjArgs {
  Geometry g;
  const double* x;        // x_n of the step (or x_K for the seed sweep)
  const double* k[5];     // k_1..k_3 of the step (k_1 is part of the stage-2 window)
  const double* y[4];     // stage inputs y_3..y_6 of the step
  const double* dt;       // device pointer to the step's dt
  const double* B0;       // B0'' (prescaled, FP64)
  const double* xbar;     // cotangent of x_{n+1}
  const double* ybar[7];  // ybar_t for t = 2..6 (index t)
  const double* ubar;     // cotangent of k_s for the field sweep of stage s < 6 (gather output)
  const double* useed;    // seed sweep: cotangent of u (may be null)
  double* Fbar;           // [9][N] cotangent of F' (row-major 3x3 per node, component-major)
  double* B0bar;          // [3][N] accumulated cotangent of B0''
  double* ybar_out;       // gather mode 0 output: ybar_t
  double* ubar_out;       // gather mode 0 output: cotangent of k_{t-1}
  double* xbar_out;       // gather modes 1, 2 output
  double gamma, seed_EM, seed_R2;
};

// Cash-Karp RK5(4) coefficients (Cash & Karp 1990): stage rows a_sj, 5th and 4th order
// weights.  (Constant tables of the integrator; compiled into the device code.)
struct CK {
  static constexpr double a[6][5] = {
      {0, 0, 0, 0, 0},
      {1.0 / 5.0, 0, 0, 0, 0},
      {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0},
      {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0, 0},
      {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0},
      {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0}};
  static constexpr double b5[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0};
  static constexpr double b4[6] = {2825.0 / 27648.0, 0.0, 18575.0 / 48384.0, 13525.0 / 55296.0,
                                   277.0 / 14336.0, 1.0 / 4.0};
};

// ------------------------------------------------------------------------------------------
// Host helpers implemented in relax.cpp
// ------------------------------------------------------------------------------------------
bool valid_config(const relax_config* c);          // every field in range
int choose_tz(const relax_config* c, int tiles_xy);  // z-chunk length
Geometry make_geometry(const relax_config* c);     // tiles, chunks and scale factors

// ------------------------------------------------------------------------------------------
// Launchers implemented in the kernel translation units
// ------------------------------------------------------------------------------------------
// stage s in 1..6; mixed selects float k / B0 storage
hipError_t launch_stage(int s, bool mixed, const SweepArgs& a, hipStream_t st);
// FP64 stage s of the forward replay of the reverse pass: stages 4 and 6 also store their
// stage input at the node into a.yrec
hipError_t launch_stage_rec(int s, const SweepArgs& a, hipStream_t st);
hipError_t launch_diagnostics(const SweepArgs& a, hipStream_t st);  // FP64 sweep of x[diag_buf]
hipError_t launch_control(Control* ctl, const double* part, const double* lam_part, int nblocks,
                          double* ring, double* dt_record, hipStream_t st);
// out6 = {E_M, R2, xi, min det F, null-guard skips, concave nodes} of a diagnostics sweep
hipError_t launch_diag_finish(const double* part, int nblocks, double dV, double* out6, hipStream_t st);
hipError_t launch_begin_chunk(Control* ctl, int target, hipStream_t st);
hipError_t launch_to_float(const double* src, float* dst, long long n, hipStream_t st);
hipError_t launch_prescale(double* B0, long long N, const double scale[3], hipStream_t st);
hipError_t launch_adj_field(int s, bool seed, const AdjArgs& a, hipStream_t st);
hipError_t launch_adj_gather(const AdjArgs& a, int mode, int stage, hipStream_t st);
hipError_t launch_fill(double* v, long long n, double val, hipStream_t st);
hipError_t launch_seg_step(Control* c2, const double* dt_record, long long n, hipStream_t st);
// out = max over nodes of |v|^2; scratch holds nscratch >= 1 doubles of per-workgroup maxima
hipError_t launch_max_norm2(const double* v, long long N, double* out, double* scratch, int nscratch,
                            hipStream_t st);

}  // namespace relax
