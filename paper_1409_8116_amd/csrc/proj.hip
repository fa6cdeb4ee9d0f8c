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

// The kernels walk rows along the contiguous axis: a block takes rows
// (c0, c1) in turn (one division per row) and its threads the elements of the
// row, so every access is coalesced and the per-element index work is an add.

// g[c] = div(vel)[c] / adt for every cell (C order).
__global__ void __launch_bounds__(PROJ_NT) proj_div_kernel(ProjDev q, double* g) {
  const int64_t n0 = q.n[0], n1 = q.n[1], n2 = q.n[2];
  for (int64_t row = blockIdx.x; row < n0 * n1; row += gridDim.x) {
    const int64_t c0 = row / n1, c1 = row - c0 * n1;
    int64_t base[3], step[3];
    for (int d = 0; d < 3; ++d) {
      base[d] = c0 * q.vs[d][0] + c1 * q.vs[d][1];
      step[d] = q.vs[d][d];
    }
    // the face above cell c along axes 0 / 1 (fixed for the row)
    const int64_t up0 = (q.ext[0] == 0 && c0 + 1 == n0) ? -(n0 - 1) * step[0] : step[0];
    const int64_t up1 = (q.ext[1] == 0 && c1 + 1 == n1) ? -(n1 - 1) * step[1] : step[1];
    const double* u0 = static_cast<const double*>(q.vel[0]);
    const double* u1 = static_cast<const double*>(q.vel[1]);
    const double* u2 = static_cast<const double*>(q.vel[2]);
    for (int64_t c2 = threadIdx.x; c2 < n2; c2 += PROJ_NT) {
      double sum = 0.0;
      if (u0) {
        const int64_t o = base[0] + c2;
        sum += (u0[o + up0] - u0[o]) * q.inv_h[0];
      }
      if (u1) {
        const int64_t o = base[1] + c2;
        sum += (u1[o + up1] - u1[o]) * q.inv_h[1];
      }
      if (u2) {
        const int64_t o = base[2] + c2;
        const int64_t up2 = (q.ext[2] == 0 && c2 + 1 == n2) ? -(n2 - 1) : 1;
        sum += (u2[o + up2] - u2[o]) * q.inv_h[2];
      }
      g[row * n2 + c2] = sum * q.inv_adt;
    }
  }
}

// Row (c0, c1) of the face array of component d < 2 (faces across rows: the
// face index is c_d; phi rows of cells f and f - 1): u_d -= adt grad_d phi.
template <typename D>
__device__ __forceinline__ void correct_row_across(const ProjDev& q, const D* phi, int d, int64_t c0, int64_t c1) {
  const int64_t n[3] = {q.n[0], q.n[1], q.n[2]};
  const int64_t cs[3] = {n[1] * n[2], n[2], 1};  // cell strides of phi
  const int ext = q.ext[d];
  const int64_t s1 = n[1] + (d == 1 ? ext : 0);  // rows of the face array along axis 1
  D* ur = static_cast<D*>(q.vel[d]) + (c0 * s1 + c1) * n[2];
  const double cu = q.adt * q.inv_h[d];
  const int64_t f = d == 0 ? c0 : c1;
  const int64_t nd = n[d];
  int64_t cc[2] = {c0, c1};
  cc[d] = f < nd ? f : nd - 1;  // the cell above the face (below it for face n)
  const D* hi = phi + cc[0] * cs[0] + cc[1] * cs[1];
  const D* lo = nullptr;
  double chi = 1.0, clo = -1.0;  // g = chi * phi[hi] + clo * phi[lo]
  if (ext == 0) {
    lo = f == 0 ? hi + (nd - 1) * cs[d] : hi - cs[d];
  } else if (f == 0) {
    if (!q.dlo[d]) return;  // Neumann face: the velocity stays
    chi = 2.0;
  } else if (f == nd) {
    if (!q.dhi[d]) return;
    chi = -2.0;
  } else {
    lo = hi - cs[d];
  }
  for (int64_t c2 = threadIdx.x; c2 < n[2]; c2 += PROJ_NT) {
    const double g = chi * double(hi[c2]) + (lo ? clo * double(lo[c2]) : 0.0);
    ur[c2] = D(double(ur[c2]) - cu * g);
  }
}

// Row (c0, c1) of the face array of component 2 (faces along the row: phi
// of the same cell row, cells f - 1 and f): u_2 -= adt grad_2 phi.
template <typename D>
__device__ __forceinline__ void correct_row_along(const ProjDev& q, const D* phi, int64_t c0, int64_t c1) {
  const int64_t n1 = q.n[1], nn = q.n[2];
  const int ext = q.ext[2];
  const int64_t nf = nn + ext;
  D* ur = static_cast<D*>(q.vel[2]) + (c0 * n1 + c1) * nf;
  const D* pr = phi + (c0 * n1 + c1) * nn;
  const double cu = q.adt * q.inv_h[2];
  for (int64_t f = threadIdx.x; f < nf; f += PROJ_NT) {
    double g;
    if (ext == 0) g = double(pr[f]) - double(pr[f == 0 ? nn - 1 : f - 1]);
    else if (f == 0) { if (!q.dlo[2]) continue; g = 2.0 * double(pr[0]); }
    else if (f == nn) { if (!q.dhi[2]) continue; g = -2.0 * double(pr[nn - 1]); }
    else g = double(pr[f]) - double(pr[f - 1]);
    ur[f] = D(double(ur[f]) - cu * g);
  }
}

// Component d (blockIdx.y < 3, when bit d of mask is set): u_d -= adt grad_d phi
// on every face; blockIdx.y == 3 (when add_p): p += phi.  When components 0
// and 1 are both corrected, the blocks of y = 0 do all of it over the union
// of the face rows of 0 and 1 (a phi row is then read once for every update
// that uses it: u, v, w and p) and the others stay idle.
template <typename D>
__global__ void __launch_bounds__(PROJ_NT) proj_correct_kernel(ProjDev q, const D* phi, int mask, int add_p) {
  const int d = int(blockIdx.y);
  const int64_t n[3] = {q.n[0], q.n[1], q.n[2]};
  const bool both = (mask & 3) == 3 && q.vel[0] && q.vel[1];
  if (both) {
    if (d != 0) return;
    const bool do_w = ((mask >> 2) & 1) && q.vel[2];
    D* p = static_cast<D*>(q.p);
    const int64_t r0 = n[0] + q.ext[0], r1 = n[1] + q.ext[1];
    for (int64_t row = blockIdx.x; row < r0 * r1; row += gridDim.x) {
      const int64_t c0 = row / r1, c1 = row - c0 * r1;
      if (c1 < n[1]) correct_row_across(q, phi, 0, c0, c1);
      if (c0 < n[0]) correct_row_across(q, phi, 1, c0, c1);
      if (c0 < n[0] && c1 < n[1]) {
        if (do_w) correct_row_along(q, phi, c0, c1);
        if (add_p) {
          const int64_t o = (c0 * n[1] + c1) * n[2];
          for (int64_t c2 = threadIdx.x; c2 < n[2]; c2 += PROJ_NT) p[o + c2] = D(double(p[o + c2]) + double(phi[o + c2]));
        }
      }
    }
    return;
  }
  if (d == 3) {
    if (!add_p) return;
    D* p = static_cast<D*>(q.p);
    const int64_t total = n[0] * n[1] * n[2];
    for (int64_t i = int64_t(blockIdx.x) * PROJ_NT + threadIdx.x; i < total; i += int64_t(gridDim.x) * PROJ_NT)
      p[i] = D(double(p[i]) + double(phi[i]));
    return;
  }
  if (!((mask >> d) & 1) || !q.vel[d]) return;
  // rows of component d's face array (axis d may have one more face)
  const int64_t s0 = n[0] + (d == 0 ? q.ext[0] : 0), s1 = n[1] + (d == 1 ? q.ext[1] : 0);
  for (int64_t row = blockIdx.x; row < s0 * s1; row += gridDim.x) {
    const int64_t c0 = row / s1, c1 = row - c0 * s1;
    if (d == 2) correct_row_along(q, phi, c0, c1);
    else correct_row_across(q, phi, d, c0, c1);
  }
}

unsigned proj_blocks(int64_t rows) {
  return unsigned(rows < 16384 ? (rows > 0 ? rows : 1) : 16384);
}

}  // namespace

hipError_t launch_proj_div(const ProjDev& q, double* g, hipStream_t s) {
  hipLaunchKernelGGL(proj_div_kernel, dim3(proj_blocks(q.n[0] * q.n[1])), dim3(PROJ_NT), 0, s, q, g);
  return hipGetLastError();
}

hipError_t launch_proj_correct(const ProjDev& q, const void* phi, int f64, int mask, int add_p, hipStream_t s) {
  // rows of the largest component (axis 0 or 1 may have one more face)
  const int64_t rows = (q.n[0] + q.ext[0]) * (q.n[1] + q.ext[1]);
  const dim3 grid(proj_blocks(rows), 4);
  if (f64)
    hipLaunchKernelGGL(proj_correct_kernel<double>, grid, dim3(PROJ_NT), 0, s, q, static_cast<const double*>(phi),
                       mask, add_p);
  else
    hipLaunchKernelGGL(proj_correct_kernel<float>, grid, dim3(PROJ_NT), 0, s, q, static_cast<const float*>(phi), mask,
                       add_p);
  return hipGetLastError();
}

}  // namespace mpois
