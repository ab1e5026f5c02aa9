// noalloc.hip -- relax_diagnostics_noalloc: the FP64 diagnostics of relax_diagnostics for
// positions and a field the caller passes directly, with no context, no workspace and no
// allocation.  Its device scratch (the control block the sweep reads, the per-workgroup
// partials of the sweep and of max |B0|^2, the final sums) is one file-scope __device__
// array of fixed size; each device the library runs on holds its own copy until the process
// ends.  Host code never uses the array's name as a device address: its address on each
// device comes from hipGetSymbolAddress, taken once per device with that device current.
#include <mutex>

#include "relax_device.h"

namespace relax {
namespace {

// workgroups of one sweep the scratch holds partials for (a 64 x 8 tile per workgroup:
// 16384 workgroups cover 2^23 nodes per z-chunk round, e.g. every grid up to 512 x 512 x nz
// with the chunk counts the library chooses)
constexpr int NA_MAX_BLOCKS = 16384;
// layout in doubles: control block, final sums, max |B0|^2, then the partial records
constexpr size_t NA_CTL = 0;
constexpr size_t NA_OUT = 128;
constexpr size_t NA_MAXB2 = NA_OUT + 8;
constexpr size_t NA_PART = 256;
constexpr size_t NA_DOUBLES = NA_PART + (size_t)NA_MAX_BLOCKS * NPART;  // 1 MiB + 2 KiB
static_assert(sizeof(Control) <= (NA_OUT - NA_CTL) * sizeof(double), "control block does not fit");

__device__ __align__(256) double scratch[NA_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_scratch[MAX_DEVICES] = {};

// address of this device's copy of `scratch` (taken once per device, with it current)
hipError_t scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

// the two control fields the diagnostics sweep reads
__global__ void na_setup_kernel(Control* ctl, double gamma, double xi_null_tau, const double* maxB2) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->gamma = gamma;
    ctl->tau_B2 = xi_null_tau * (*maxB2);
  }
}

}  // namespace
}  // namespace relax

using namespace relax;

extern "C" int relax_diagnostics_noalloc(const relax_config* cfg, const double* d_x, const double* d_B0,
                                         void* hip_stream, relax_diag* out) {
  if (!cfg || !d_x || !d_B0 || !out || !valid_config(cfg)) return RELAX_E_ARG;
  const Geometry g = make_geometry(cfg);
  if (g.nblocks > NA_MAX_BLOCKS) return RELAX_E_SPACE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  double* base = nullptr;
  if (scratch_ptr(&base) != hipSuccess) return RELAX_E_HIP;
  Control* ctl = reinterpret_cast<Control*>(base + NA_CTL);
  double* d_out = base + NA_OUT;
  double* d_maxB2 = base + NA_MAXB2;
  double* d_part = base + NA_PART;

  SweepArgs a{};
  a.g = g;
  a.x[0] = a.x[1] = d_x;
  a.B0 = d_B0;  // unscaled: the sweep applies B0'' = 4 h_b h_c B0 as it loads it
  for (int m = 0; m < 3; m++) a.b0_mul[m] = g.b0scale[m];
  a.ctl = ctl;
  a.part = d_part;
  a.diag_buf = 0;

  // max |B0|^2 of the caller's field (the xi null guard), the two control fields, the FP64
  // diagnostics sweep and its fixed-order final reduction
  if (launch_max_norm2(d_B0, g.N, d_maxB2, d_part, NA_MAX_BLOCKS * NPART, st) != hipSuccess) return RELAX_E_HIP;
  hipLaunchKernelGGL(na_setup_kernel, dim3(1), dim3(64), 0, st, ctl, cfg->gamma, cfg->xi_null_tau, d_maxB2);
  if (hipGetLastError() != hipSuccess) return RELAX_E_HIP;
  if (launch_diagnostics(a, st) != hipSuccess) return RELAX_E_HIP;
  if (launch_diag_finish(d_part, g.nblocks, g.dV, d_out, st) != hipSuccess) return RELAX_E_HIP;
  double d[6];
  if (hipMemcpyAsync(d, d_out, sizeof(d), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return RELAX_E_HIP;
  out->t = 0.0;
  out->dt = cfg->dt0;
  out->E_M = d[0];
  out->R2 = d[1];
  out->xi = d[2];
  out->min_det = d[3];
  out->Lambda = 0.0;
  out->rejects = 0;
  out->concave = (int)d[5];
  return RELAX_OK;
}
