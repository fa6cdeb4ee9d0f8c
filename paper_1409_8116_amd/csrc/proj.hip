// Kernels of the projection step around the Poisson solve (incompressible
// flow on the staggered MAC grid, paper Section 5.1): the divergence of the
// predicted velocity as a right-hand side, and the correction
// u -= alpha dt grad phi on the faces together with p += phi.  The line
// passes fuse the first into their loads and the correction of the
// last-axis component (and p) into their stores; these kernels cover the
// other components, and all of it for plans whose solve needs the right-hand
// side as an array (FP32 solve with FP64 refinement).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mpois {

namespace {

constexpr int PROJ_NT = 256;

// Index arithmetic in 32 bits when the array allows it.
template <typename I>
__device__ __forceinline__ void unflatten(I i, const I s[3], I c[3]) {
  c[2] = i % s[2];
  const I r = i / s[2];
  c[1] = r % s[1];
  c[0] = r / s[1];
}

// g[c] = div(vel)[c] / adt for every cell (C order).
template <typename I>
__device__ void div_cells(const ProjDev& q, double* g) {
  const I s[3] = {I(q.n[0]), I(q.n[1]), I(q.n[2])};
  const I total = s[0] * s[1] * s[2];
  for (I i = I(blockIdx.x) * PROJ_NT + threadIdx.x; i < total; i += I(gridDim.x) * PROJ_NT) {
    I c[3];
    unflatten(i, s, c);
    double sum = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double* u = static_cast<const double*>(q.vel[d]);
      if (!u) continue;
      const I vd = I(q.vs[d][d]);
      const I o = c[0] * I(q.vs[d][0]) + c[1] * I(q.vs[d][1]) + c[2] * I(q.vs[d][2]);
      const I up = (q.ext[d] == 0 && c[d] + 1 == s[d]) ? o - (s[d] - 1) * vd : o + vd;
      sum += (u[up] - u[o]) * q.inv_h[d];
    }
    g[i] = sum * q.inv_adt;
  }
}

__global__ void __launch_bounds__(PROJ_NT) proj_div_kernel(ProjDev q, double* g, int wide) {
  if (wide) div_cells<int64_t>(q, g);
  else div_cells<uint32_t>(q, g);
}

// Component d (blockIdx.y < 3, when bit d of mask is set): u_d -= adt grad_d phi
// on every face; blockIdx.y == 3 (when add_p): p += phi.
template <typename D, typename I>
__device__ void correct(const ProjDev& q, const D* phi, int mask, int add_p) {
  const int d = int(blockIdx.y);
  const I cs[3] = {I(q.n[1] * q.n[2]), I(q.n[2]), 1};  // cell strides of phi
  if (d == 3) {
    if (!add_p) return;
    D* p = static_cast<D*>(q.p);
    const I total = I(q.n[0] * q.n[1] * q.n[2]);
    for (I i = I(blockIdx.x) * PROJ_NT + threadIdx.x; i < total; i += I(gridDim.x) * PROJ_NT)
      p[i] = D(double(p[i]) + double(phi[i]));
    return;
  }
  if (!((mask >> d) & 1) || !q.vel[d]) return;
  D* u = static_cast<D*>(q.vel[d]);
  const I n = I(q.n[d]);
  const int ext = q.ext[d];
  I s[3] = {I(q.n[0]), I(q.n[1]), I(q.n[2])};
  s[d] += I(ext);
  const I total = s[0] * s[1] * s[2];
  const double cu = q.adt * q.inv_h[d];
  for (I i = I(blockIdx.x) * PROJ_NT + threadIdx.x; i < total; i += I(gridDim.x) * PROJ_NT) {
    I c[3];
    unflatten(i, s, c);
    const I f = c[d];
    c[d] = f < n ? f : n - 1;  // cell above the face (below it for face n)
    const I o = c[0] * cs[0] + c[1] * cs[1] + c[2] * cs[2];
    double g;
    if (ext == 0) {
      g = double(phi[o]) - double(phi[f == 0 ? o + (n - 1) * cs[d] : o - cs[d]]);
    } else if (f == 0) {
      if (!q.dlo[d]) continue;  // Neumann face: no flux, the velocity stays
      g = 2.0 * double(phi[o]);
    } else if (f == n) {
      if (!q.dhi[d]) continue;
      g = -2.0 * double(phi[o]);
    } else {
      g = double(phi[o]) - double(phi[o - cs[d]]);
    }
    u[i] = D(double(u[i]) - cu * g);
  }
}

template <typename D>
__global__ void __launch_bounds__(PROJ_NT) proj_correct_kernel(ProjDev q, const D* phi, int mask, int add_p,
                                                               int wide) {
  if (wide) correct<D, int64_t>(q, phi, mask, add_p);
  else correct<D, uint32_t>(q, phi, mask, add_p);
}

// Largest element count among the velocity components and the cells.
int64_t proj_extent(const ProjDev& q) {
  int64_t m = q.n[0] * q.n[1] * q.n[2];
  for (int d = 0; d < 3; ++d) {
    int64_t s[3] = {q.n[0], q.n[1], q.n[2]};
    s[d] += q.ext[d];
    m = s[0] * s[1] * s[2] > m ? s[0] * s[1] * s[2] : m;
  }
  return m;
}

unsigned proj_blocks(int64_t count) {
  const int64_t b = (count + PROJ_NT - 1) / PROJ_NT;
  return unsigned(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

hipError_t launch_proj_div(const ProjDev& q, double* g, hipStream_t s) {
  const int64_t ext = proj_extent(q);
  hipLaunchKernelGGL(proj_div_kernel, dim3(proj_blocks(q.n[0] * q.n[1] * q.n[2])), dim3(PROJ_NT), 0, s, q, g,
                     int(ext >= (int64_t(1) << 31)));
  return hipGetLastError();
}

hipError_t launch_proj_correct(const ProjDev& q, const void* phi, int f64, int mask, int add_p, hipStream_t s) {
  const int64_t ext = proj_extent(q);
  const dim3 grid(proj_blocks(ext), 4);
  const int wide = int(ext >= (int64_t(1) << 31));
  if (f64)
    hipLaunchKernelGGL(proj_correct_kernel<double>, grid, dim3(PROJ_NT), 0, s, q, static_cast<const double*>(phi),
                       mask, add_p, wide);
  else
    hipLaunchKernelGGL(proj_correct_kernel<float>, grid, dim3(PROJ_NT), 0, s, q, static_cast<const float*>(phi), mask,
                       add_p, wide);
  return hipGetLastError();
}

}  // namespace mpois
