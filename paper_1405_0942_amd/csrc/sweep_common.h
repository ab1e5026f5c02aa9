// sweep_common.h -- device helpers shared by the forward stage sweeps (stage.hip) and the
// reverse sweeps (adjoint.hip): index resolution on line-tied and periodic axes, raw buffer
// accesses with masked-off lanes, the XCD-aware tile order, the 3x3 determinant and a
// Newton-refined reciprocal.  Internal to the library.
#pragma once

#include "relax_device.h"

namespace relax {

__device__ __forceinline__ int floordiv(int a, int n) { return a >= 0 ? a / n : -((-a + n - 1) / n); }
// p mod 3 in [0, 3) for p >= -3072 (plane indices reach at most three planes below 0)
__device__ __forceinline__ int mod3(int p) { return (int)((unsigned)(p + 3072) % 3u); }

// One axis of a neighbour index: the in-range index, the number of periods wrapped (periodic
// axes), and whether the node exists (line-tied axes end at the boundary nodes).
struct AxisIdx {
  int i;
  int w;
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

// resolve() without divisions, exact for v in [-n, 2n): the plane indices of a z march lie
// within three planes of [0, n) and n >= 4.  Other v give a wrong but in-range index.
__device__ __forceinline__ AxisIdx resolve_near(int v, int n, int bc) {
  if (bc == BC_PERIODIC) {
    const int w = v < 0 ? -1 : (v >= n ? 1 : 0);
    return AxisIdx{min(max(v - w * n, 0), n - 1), w, true};
  }
  return resolve(v, n, bc);
}

// ---- buffer access --------------------------------------------------------------------------
// Element index of a masked-off lane: scaled by the element size it lands at or past the
// record count of every plane (a plane holds fewer than 2^28 nodes), so its load returns 0 and
// its store is dropped.
constexpr unsigned IE = 1u << 28;
constexpr int RSRC_WORD3 = 0x00020000;  // raw (untyped) buffer resource, gfx9 encoding
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// cache policy of the single-use accesses (node-wise loads and all stores): nt, non-temporal.
// The stencilled loads keep the default so that neighbouring tiles find their halo lines in L2.
constexpr int CPOL_STREAM = 2;

// resource for one component plane [base, base + nxy)
template <typename V>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const V* base, unsigned nxy) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<V*>(base), 0, (int)(nxy * sizeof(V)), RSRC_WORD3);
}
template <typename V, int CP = 0>
__device__ __forceinline__ V bload(__amdgpu_buffer_rsrc_t r, unsigned e) {
  if constexpr (sizeof(V) == 8)
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, (int)(e * 8u), 0, CP));
  else
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, (int)(e * 4u), 0, CP));
}
template <typename V>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned e, V v) {
  if constexpr (sizeof(V) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)(e * 8u), 0, CPOL_STREAM);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)(e * 4u), 0, CPOL_STREAM);
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

}  // namespace relax
