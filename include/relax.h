/*
 * relax.h -- C ABI of the MI355X (gfx950) Lagrangian mimetic magneto-frictional relaxation
 * step (Candelaresi, Pontin & Hornig, "Mimetic Methods for Lagrangian Relaxation of
 * Magnetic Fields").
 *
 * The state is the Lagrangian map x(X, t) sampled on a logically rectangular, node-centred
 * grid of reference positions X (Sec. 1, eq. "x integration").  The field is frozen in:
 * at every node B = F B0 / det F with F = dx/dX (Sec. 2.1, eq. "B transformation").  The
 * current J = curl B is the Stokes-loop mimetic operator of Sec. 2.2 (eqs. "current
 * discrete", "four surfaces", "sum of triangles", "current matrix equation") and the
 * velocity is the magneto-frictional u = gamma J x B (Sec. 1, eq. "magneto friction").
 * x is advanced by the fifth-order adaptive Cash-Karp Runge-Kutta method with the
 * step-size rule of Sec. 2.4 (eq. "time stepping").  Boundaries are line-tied or
 * periodic with shifted ghost positions (Sec. 2.5).
 *
 * Conventions
 *  - Fields are structure-of-arrays FP64 [3][nz][ny][nx], x fastest: component c of node
 *    (i, j, k) is at c*N + (k*ny + j)*nx + i with N = nx*ny*nz.
 *  - Pointers named d_* are device pointers (HIP), owned by the caller.  The library never
 *    allocates device memory: all its device state lives in the caller's workspace.
 *  - hip_stream is a hipStream_t (may be NULL for the default stream).  All work is
 *    enqueued on it; a call returns after the host copies it documents.
 *  - Every function returns RELAX_OK (0) or a negative RELAX_E_* code and never throws.
 *    After RELAX_E_FOLD, RELAX_E_DT, RELAX_E_NAN or RELAX_E_HIP a context is failed: every
 *    further call except relax_get_state, relax_set_state, relax_last_error and
 *    relax_destroy returns RELAX_E_STATE.
 *  - Calls on one context must not overlap; different contexts are independent.
 */
#ifndef RELAX_H
#define RELAX_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RELAX_OK = 0,
  RELAX_E_ARG = -1,   /* invalid argument or configuration */
  RELAX_E_HIP = -2,   /* a HIP runtime call failed */
  RELAX_E_FOLD = -3,  /* min det F <= 0: folded grid (the paper's breakdown, Sec. 4.4) */
  RELAX_E_DT = -4,    /* step rejected below dt_min (dt collapse, Sec. 4.4) */
  RELAX_E_NAN = -5,   /* non-finite energy, residual or error estimate */
  RELAX_E_STATE = -6, /* context failed earlier, or no recorded trajectory */
  RELAX_E_SPACE = -7  /* workspace too small */
};

enum { RELAX_LINE_TIED = 0, RELAX_PERIODIC = 1 };
enum { RELAX_FP64 = 0, RELAX_FP32_MIXED = 1 };
enum { RELAX_CURL_NN = 0, RELAX_CURL_NNN = 1 };

typedef struct {
  int n[3];             /* nodes along x, y, z; each >= 4, n[0] * n[1] < 2^28 */
  double h[3];          /* reference spacing dX, dY, dZ (> 0).  Periodic period P_a = n_a h_a */
  int bc[3];            /* per axis RELAX_LINE_TIED or RELAX_PERIODIC (Sec. 2.5) */
  int precision;        /* RELAX_FP64, or RELAX_FP32_MIXED: stage vectors, B0 copy and the
                           stencil past the Jacobian in FP32; positions, det F, the energy and
                           residual reductions and the step control in FP64 */
  double gamma;         /* friction coefficient (the paper uses 1, Sec. 2.1) */
  double dt0;           /* first step size (> 0) */
  double dt_min;        /* a rejected step below this fails with RELAX_E_DT */
  double tol;           /* Lambda_0: bound on the max-norm error estimate of x per step */
  int adaptive;         /* 1: the step-size rule of Sec. 2.4; 0: fixed dt = dt0 */
  int record;           /* 1: keep the dt of every step and x every checkpoint_every steps
                           for relax_backward */
  int checkpoint_every; /* checkpoint interval c (>= 1) when record = 1 */
  double xi_null_tau;   /* xi skips nodes with |B|^2 <= xi_null_tau * max |B0|^2 (e.g. 1e-12) */
  double safety;        /* (0, 1]: factor on the new step of the rule of Sec. 2.4 (rejected and
                           grown steps).  1 is the rule as the paper prints it; there a
                           stability-limited run near equilibrium, where Lambda barely depends
                           on dt, can retry a rejected step with nearly the same dt for a very
                           long time.  0.9 (the Numerical Recipes value) avoids that. */
  int curl;             /* RELAX_CURL_NN: the current from loops over the four in-plane nearest
                           neighbours (Sec. 2.2), the default; RELAX_CURL_NNN: loops over the
                           octilateral of the eight in-plane ring neighbours (Sec. 2.3; FP64
                           only, no relax_backward) */
} relax_config;

/* Per accepted step, evaluated at the state the step starts from (pre-step). */
typedef struct {
  double t;       /* time of the state */
  double dt;      /* accepted step size */
  double E_M;     /* magnetic energy 1/2 sum zeta |B|^2 det F dX dY dZ (eq. "magnetic energy") */
  double xi;      /* max over interior nodes of |J x B| / |B|^2 (Sec. 4.1) */
  double R2;      /* 1/2 sum_interior det F |J x B|^2 dX dY dZ (smooth force residual) */
  double Lambda;  /* error estimate max |x5 - x4| of the accepted attempt */
  double min_det; /* min det F over all nodes */
  int rejects;    /* rejected attempts before acceptance */
  int concave;    /* nodes that are not convex (Sec. 3.2.3, eq. "convexity": some trihedron of
                     edge vectors to neighbours has the wrong determinant sign; trihedra beyond
                     a line-tied face are not formed).  Evaluated by relax_diagnostics only;
                     0 in the per-step records of relax_step. */
} relax_diag;

/* Bytes of device workspace a context with this configuration needs (the state of Sec. 1 and
 * the Runge-Kutta stage vectors of Sec. 2.4, plus checkpoints for relax_backward).  K_record is the
 * number of steps relax_backward may later differentiate through (0 if record = 0).
 * Returns 0 for an invalid configuration. */
size_t relax_workspace_bytes(const relax_config* cfg, int K_record);

/* Create a context (Sec. 1: the state is the map x(X, t) on the grid of reference positions X,
 * with the field B0 = B(X, 0) frozen in through eq. "B transformation" of Sec. 2.1; boundary
 * kinds of Sec. 2.5).  d_x0 (initial positions) and d_B0 (initial field at the nodes,
 * B(X, 0)) are [3][nz][ny][nx] FP64 device arrays; they are copied, so the caller may
 * free them afterwards.  d_workspace (>= relax_workspace_bytes(cfg, K_record) bytes,
 * 256-byte aligned) belongs to the context until relax_destroy.  A folded x0 returns
 * RELAX_E_FOLD and no context.  Synchronises hip_stream once. */
int relax_init(const relax_config* cfg, int K_record, const double* d_x0, const double* d_B0,
               void* d_workspace, size_t workspace_bytes, void* hip_stream, void** out_ctx);

/* Advance by K accepted steps of the fifth-order adaptive Cash-Karp Runge-Kutta method with
 * the step-size rule of Sec. 2.4 (eq. "time stepping"; fixed dt = dt0 if cfg->adaptive = 0)
 * applied to dx/dt = u (Sec. 1, eqs. "x integration", "magneto friction").  Rejected attempts
 * are redone inside.  If
 * host_diag is not NULL it receives K entries (host memory), one per accepted step.
 * On an error the steps completed before it are kept and reported in *steps_done (may be
 * NULL).  Blocks until the steps are done. */
int relax_step(void* ctx, int K, relax_diag* host_diag, int* steps_done);

/* FP64 diagnostics sweep of the current positions (also for a mixed-precision context):
 * fills t, dt (next step size), E_M (Sec. 3.2.4, eq. "magnetic energy"), xi (Sec. 4.1), R2,
 * min_det and concave (Sec. 3.2.3); Lambda and rejects are 0. */
int relax_diagnostics(void* ctx, relax_diag* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc) and hold no context: the diagnostics of
 * relax_diagnostics for positions d_x and initial field d_B0 given directly ([3][nz][ny][nx]
 * FP64 device arrays, read only), with the configuration cfg (n, h, bc, gamma, xi_null_tau;
 * dt0 is reported as dt, t as 0).  The result equals relax_diagnostics of a context created
 * by relax_init(cfg, ..., d_x, d_B0, ...).  No allocation: the call's device scratch is a
 * fixed array of the library (1 MiB per device, held until the process ends), enough for
 * sweeps of at most 16384 workgroups of 64 x 8 nodes (for example every grid of up to
 * 512 x 512 x 512 nodes); larger grids return RELAX_E_SPACE before any GPU work.  Calls on
 * one device share that scratch: calls that overlap on one device (several host threads, or
 * several streams) race and must not be made.  Blocks until done. */
int relax_diagnostics_noalloc(const relax_config* cfg, const double* d_x, const double* d_B0, void* hip_stream,
                              relax_diag* out);

/* Velocity u = gamma J x B of the current positions (Sec. 1, eq. "magneto friction", with
 * J the mimetic current of Sec. 2.2), evaluated in FP64 (also for a mixed-precision
 * context) into d_u_out (device, [3][nz][ny][nx], overwritten; zero on line-tied faces).
 * Blocks until done. */
int relax_velocity(void* ctx, double* d_u_out);

/* The pulled-back field B = F B0 / det F (Sec. 2.1, eq. "B transformation") and the mimetic
 * current J (Sec. 2.2) of the current positions, evaluated in FP64 (also for a mixed-precision
 * context) into d_B_out and d_J_out (device, [3][nz][ny][nx], overwritten).  J is zero on
 * line-tied faces, where the loops of Sec. 2.2 are not closed.  Either pointer may be NULL.
 * Blocks until done. */
int relax_fields(void* ctx, double* d_B_out, double* d_J_out);

/* Breakdown monitors of the current positions, per node ([nz][ny][nx], device, overwritten):
 * d_alpha_out (FP64) receives alpha* = J.B / |B|^2 (Sec. 3.2.1; constant along field lines in a
 * force-free state; 0 where B = 0 and on line-tied faces, where J is 0), with B and J as
 * relax_fields gives them; d_kappa_out (int32) receives the convexity of Sec. 3.2.3
 * (eq. "convexity"): +1 if every trihedron of edge vectors to the neighbours
 * x(i +- 1, j, k), x(i, j +- 1, k), x(i, j, k +- 1) has the determinant sign of its
 * orientation, else -1 (trihedra beyond a line-tied face are not formed; the count of -1 nodes
 * is relax_diag.concave).  Either pointer may be NULL.  Blocks until done. */
int relax_monitors(void* ctx, double* d_alpha_out, int* d_kappa_out);

/* Reverse-mode gradient (the transpose of the step of relax_step: Sec. 2.1 pull-back, Sec. 2.2
 * mimetic current, Sec. 2.4 Runge-Kutta stages) through the recorded trajectory, with its dt
 * sequence held fixed (record = 1):
 * d(seed_EM * E_M(x_K) + seed_R2 * R2(x_K)) / d(x0, B0), where x_K is the current state
 * and x0 the state at init / relax_set_state.  d_grad_x0, d_grad_B0: [3][nz][ny][nx] FP64
 * device arrays (overwritten).  Returns RELAX_E_STATE if nothing was recorded. */
int relax_backward(void* ctx, double seed_EM, double seed_R2, double* d_grad_x0, double* d_grad_B0);

/* Copy the current positions x(X, t) (Sec. 1, the Lagrangian map) to d_x_out (device,
 * [3][nz][ny][nx] FP64) and read t and the next step size of the rule of Sec. 2.4; any output
 * may be NULL. */
int relax_get_state(void* ctx, double* d_x_out, double* t, double* dt);

/* Replace the positions x(X, t) (Sec. 1; device array, copied), t and dt; clears a failed
 * state and the recorded trajectory.  A folded state (some det F <= 0, the breakdown of
 * Sec. 4.4) returns RELAX_E_FOLD. */
int relax_set_state(void* ctx, const double* d_x_in, double t, double dt);

/* Per-kernel timing.  Returns the totals accumulated since the previous call (then resets
 * them) and switches timing on (on = 1) or off (0).  While on, relax_step brackets each
 * kernel launch with HIP events on hip_stream.  ms_out[7] / launches_out[7] (host, may be
 * NULL): index 0..5 = the six Runge-Kutta stage sweeps, 6 = the step-control kernel. */
int relax_profile(void* ctx, int on, double* ms_out, long long* launches_out);

/* Measurement aid, not part of the method: the bandwidth a plain streaming kernel with the
 * stage sweeps' element width reaches (one FP64 element per lane, non-temporal loads and
 * stores, grid-stride over n elements).  kind 0: out = in (copy, one read and one write per
 * element); 1: read in only (out[0] is left as it is); 2: out = in[0:n] + in[n:2n] (two reads, one
 * write); 3: out = the sum of four consecutive input arrays of n (four reads, one write).
 * d_in holds n, n, 2n or 4n doubles and d_out n doubles (device).  Runs once untimed, then
 * reps times; *ms_out (host) receives the mean duration of one run in milliseconds
 * (HIP events on hip_stream).  Blocks until done. */
int relax_stream_probe(int kind, const double* d_in, double* d_out, long long n, int reps, void* hip_stream,
                       double* ms_out);

/* Short English text of a status code (static storage). */
const char* relax_strerror(int code);

/* Text of the last error recorded on this context ("" if none). */
const char* relax_last_error(void* ctx);

/* Release the context (host memory only; the workspace goes back to the caller). */
void relax_destroy(void* ctx);

#ifdef __cplusplus
}
#endif

#endif /* RELAX_H */
