// dm_order.hpp -- the probe-first order of the overlap projection: the order
// in which Eqs. 4-5 are written, before the swap of the probe and object
// updates that Section III describes (the swap to object first is what lets
// a batch's object embedding overlap the next batch's view update).  Probe
// first, the probe (Eq. 4) is updated from the new views and the current
// object, and the object (Eq. 5) then from the new views and the new probe;
// the object gather therefore needs per-view numerators
// sum_k conj(P'_k) psi'_{j,k} formed with the new probe, which this kernel
// writes over the ones the view kernels formed with the old probe.
#pragma once
#include <hip/hip_runtime.h>

#include "dm_kernels.hpp"

namespace dmk {

// grid (total views, ceil(F * F / 256), L); block 256 pixels of one view and
// one object mode l (frames l M .. l M + M - 1 of the view)
__global__ __launch_bounds__(256) void k_view_numerators(const ScanDev* __restrict__ scans,
                                                         const int2* __restrict__ vmap, int M,
                                                         int FF) {
  const int2 vm = vmap[blockIdx.x];
  const ScanDev& sc = scans[vm.x];
  const int j = vm.y;
  const int L = sc.L, l = blockIdx.z;
  const int p = blockIdx.y * 256 + threadIdx.x;
  if (p >= FF) return;
  const float2* __restrict__ psi = sc.psi + ((size_t)j * L + l) * M * FF + p;
  const float2* __restrict__ P = sc.P + p;
  float2 v[8], q[8];
  float2 acc = make_float2(0.f, 0.f);
  // modes in batches of eight loads before their products
  for (int k0 = 0; k0 < M; k0 += 8) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      v[k] = (k0 + k < M) ? psi[(size_t)(k0 + k) * FF] : make_float2(0.f, 0.f);
      q[k] = (k0 + k < M) ? P[(size_t)(k0 + k) * FF] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) acc = cadd(acc, cmulc(q[k], v[k]));
  }
  sc.opart[((size_t)j * L + l) * FF + p] = acc;
}

}  // namespace dmk
