// control.hip -- device-side step control and the small set-up / reduction kernels.
//
// The control kernel closes one Cash-Karp attempt without a host round trip: it reduces
// the per-workgroup partials of the stage sweeps in a fixed order (deterministic), checks
// for breakdown, and applies the step-size rule of Sec. 2.4 (eq. "time stepping"):
//     dt' = dt |Lambda_0 / Lambda|^{0.2}
//     Lambda >  Lambda_0       -> reject, retry from x_n with dt'
//     Lambda <  Lambda_0 / 2   -> accept, continue with dt'
//     otherwise                -> accept, keep dt
// (Lambda == 0 grows the step 5x.)  On acceptance it records the step's diagnostics in
// the device ring and swaps the position buffers.
#include "relax_device.h"

namespace relax {
namespace {

constexpr int CT = 256;  // control workgroup size

__device__ __forceinline__ double max_nan(double a, double b) { return (b > a || b != b) ? b : a; }
__device__ __forceinline__ double min_nan(double a, double b) { return (b < a || b != b) ? b : a; }

// status codes (the values of include/relax.h)
constexpr int E_FOLD = -3, E_DT = -4, E_NAN = -5;

__global__ __launch_bounds__(CT) void control_kernel(Control* ctl, const double* __restrict__ part,
                                                      const double* __restrict__ lam_part, int nblocks,
                                                      double* __restrict__ ring, double* __restrict__ dt_record) {
  if (ctl->status != 0 || ctl->accepted >= ctl->target) return;
  const int tid = threadIdx.x;
  const bool fresh = (ctl->need_k1 != 0);
  __shared__ double sE[CT], sR[CT], sX[CT], sM[CT], sZ[CT], sL[CT];
  double E = 0, R = 0, X = 0, M = INFINITY, Z = 0, L = 0;
  for (int b = tid; b < nblocks; b += CT) {
    if (fresh) {
      const double* p = part + (long long)b * NPART;
      E += p[0];
      R += p[1];
      X = max_nan(X, p[2]);
      M = min_nan(M, p[3]);
      Z += p[4];
    }
    L = max_nan(L, lam_part[b]);
  }
  sE[tid] = E;
  sR[tid] = R;
  sX[tid] = X;
  sM[tid] = M;
  sZ[tid] = Z;
  sL[tid] = L;
  __syncthreads();
  for (int s = CT / 2; s > 0; s >>= 1) {
    if (tid < s) {
      sE[tid] += sE[tid + s];
      sR[tid] += sR[tid + s];
      sX[tid] = max_nan(sX[tid], sX[tid + s]);
      sM[tid] = min_nan(sM[tid], sM[tid + s]);
      sZ[tid] += sZ[tid + s];
      sL[tid] = max_nan(sL[tid], sL[tid + s]);
    }
    __syncthreads();
  }
  if (tid != 0) return;

  Control& c = *ctl;
  if (fresh) {
    c.E = 0.5 * sE[0] * c.dV;
    c.R2 = 0.5 * sR[0] * c.dV;
    c.xi = sX[0];
    c.min_det = sM[0];
    c.nulls = sZ[0];
    c.need_k1 = 0;
    if (c.min_det != c.min_det) {
      c.status = E_NAN;
      return;
    }
    if (!(c.min_det > 0.0)) {
      c.status = E_FOLD;
      return;
    }
    if (!isfinite(c.E) || !isfinite(c.R2)) {
      c.status = E_NAN;
      return;
    }
  }
  const double lam = sL[0];
  c.lambda = lam;
  if (lam != lam || isinf(lam)) {
    c.status = E_NAN;
    return;
  }
  const double dt = c.dt;
  double dt_next = dt;
  bool accept = true;
  if (c.adaptive) {
    const double dtp = (lam > 0.0) ? c.safety * dt * pow(fabs(c.tol / lam), 0.2) : 5.0 * dt;
    if (lam > c.tol) {
      accept = false;
      dt_next = dtp;
    } else {
      dt_next = (lam < 0.5 * c.tol) ? dtp : dt;
    }
  }
  if (!accept) {
    c.rejects += 1;
    c.dt = dt_next;
    if (dt_next < c.dt_min) c.status = E_DT;
    return;
  }
  double* e = ring + (long long)c.accepted * 8;
  e[0] = c.t;
  e[1] = dt;
  e[2] = c.E;
  e[3] = c.xi;
  e[4] = c.R2;
  e[5] = lam;
  e[6] = c.min_det;
  e[7] = (double)c.rejects;
  if (c.record && dt_record && c.steps_total < c.record_cap) dt_record[c.steps_total] = dt;
  c.t += dt;
  c.dt = dt_next;
  c.cur = 1 - c.cur;
  c.accepted += 1;
  c.steps_total += 1;
  c.rejects = 0;
  c.need_k1 = 1;
}

// final reduction of a diagnostics sweep: out = {sum E, sum R2, max xi, min det, nulls}
__global__ __launch_bounds__(CT) void diag_finish_kernel(const double* __restrict__ part, int nblocks, double dV,
                                                          double* __restrict__ out) {
  const int tid = threadIdx.x;
  __shared__ double sE[CT], sR[CT], sX[CT], sM[CT], sZ[CT], sC[CT];
  double E = 0, R = 0, X = 0, M = INFINITY, Z = 0, Cc = 0;
  for (int b = tid; b < nblocks; b += CT) {
    const double* p = part + (long long)b * NPART;
    E += p[0];
    R += p[1];
    X = max_nan(X, p[2]);
    M = min_nan(M, p[3]);
    Z += p[4];
    Cc += p[5];
  }
  sE[tid] = E;
  sR[tid] = R;
  sX[tid] = X;
  sM[tid] = M;
  sZ[tid] = Z;
  sC[tid] = Cc;
  __syncthreads();
  for (int s = CT / 2; s > 0; s >>= 1) {
    if (tid < s) {
      sE[tid] += sE[tid + s];
      sR[tid] += sR[tid + s];
      sX[tid] = max_nan(sX[tid], sX[tid + s]);
      sM[tid] = min_nan(sM[tid], sM[tid + s]);
      sZ[tid] += sZ[tid + s];
      sC[tid] += sC[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = 0.5 * sE[0] * dV;
    out[1] = 0.5 * sR[0] * dV;
    out[2] = sX[0];
    out[3] = sM[0];
    out[4] = sZ[0];
    out[5] = sC[0];
  }
}

__global__ void begin_chunk_kernel(Control* ctl, int target) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->accepted = 0;
    ctl->target = target;
  }
}

__global__ void to_float_kernel(const double* __restrict__ s, float* __restrict__ d, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    d[i] = (float)s[i];
}

// component-wise scaling of a [3][N] field in place
__global__ void prescale_kernel(double* __restrict__ v, long long N, double s0, double s1, double s2) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    v[i] *= s0;
    v[i + N] *= s1;
    v[i + 2 * N] *= s2;
  }
}

// max over nodes of |v|^2 of a [3][N] field, in two passes (used once at set-up): each
// workgroup reduces a grid-stride share into part[blockIdx.x], then one workgroup reduces
// the partials (a max, so the result does not depend on the order)
__global__ __launch_bounds__(CT) void max_norm2_part_kernel(const double* __restrict__ v, long long N,
                                                             double* __restrict__ part) {
  __shared__ double s[CT];
  double m = 0.0;
  for (long long i = (long long)blockIdx.x * CT + threadIdx.x; i < N; i += (long long)gridDim.x * CT) {
    const double a = v[i], b = v[i + N], c = v[i + 2 * N];
    m = max_nan(m, a * a + b * b + c * c);
  }
  s[threadIdx.x] = m;
  __syncthreads();
  for (int k = CT / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] = max_nan(s[threadIdx.x], s[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(CT) void max_reduce_kernel(const double* __restrict__ part, int n,
                                                        double* __restrict__ out) {
  __shared__ double s[CT];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += CT) m = max_nan(m, part[i]);
  s[threadIdx.x] = m;
  __syncthreads();
  for (int k = CT / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] = max_nan(s[threadIdx.x], s[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

}  // namespace

hipError_t launch_control(Control* ctl, const double* part, const double* lam_part, int nblocks, double* ring,
                          double* dt_record, hipStream_t st) {
  hipLaunchKernelGGL(control_kernel, dim3(1), dim3(CT), 0, st, ctl, part, lam_part, nblocks, ring, dt_record);
  return hipGetLastError();
}

hipError_t launch_diag_finish(const double* part, int nblocks, double dV, double* out6, hipStream_t st) {
  hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(CT), 0, st, part, nblocks, dV, out6);
  return hipGetLastError();
}

hipError_t launch_begin_chunk(Control* ctl, int target, hipStream_t st) {
  hipLaunchKernelGGL(begin_chunk_kernel, dim3(1), dim3(64), 0, st, ctl, target);
  return hipGetLastError();
}

hipError_t launch_to_float(const double* src, float* dst, long long n, hipStream_t st) {
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(to_float_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_prescale(double* B0, long long N, const double scale[3], hipStream_t st) {
  long long blocks = (N + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(prescale_kernel, dim3((unsigned)blocks), dim3(256), 0, st, B0, N, scale[0], scale[1], scale[2]);
  return hipGetLastError();
}

hipError_t launch_max_norm2(const double* v, long long N, double* out, double* scratch, int nscratch,
                            hipStream_t st) {
  long long blocks = (N + CT - 1) / CT;
  if (blocks > nscratch) blocks = nscratch;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(max_norm2_part_kernel, dim3((unsigned)blocks), dim3(CT), 0, st, v, N, scratch);
  hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(CT), 0, st, scratch, (int)blocks, out);
  return hipGetLastError();
}

}  // namespace relax
