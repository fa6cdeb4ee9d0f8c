// Auxiliary kernels: FP64 stencil residual with the zero-mode reductions, the
// fixed-order finalisation of block partial sums, and a zero fill.
//
// resid_kernel computes g - m_g - (L_h - sigma) phi for the second-order
// stencil of Eq. (FD2) with the boundary closure of each end of each axis (and
// the Helmholtz shift sigma), and block partial sums of
// w phi, w g, r^2 and (g - m_g)^2, where w is the gauge / compatibility weight
// (1/2 on the end nodes of vertex-grid Neumann axes, 1 elsewhere).  Without
// phi it only forms the sums of g.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mpois {

// ----------------------------------------------------------------------------- residual
// Gauge weight of node i: 1/2 on an end node closed by a vertex-Neumann mirror
// (only singular problems use it: Neumann on both faces of such axes).
__device__ __forceinline__ double axis_weight(int clo, int chi, int64_t i, int64_t n) {
  return ((clo == C_NV && i == 0) || (chi == C_NV && i == n - 1)) ? 0.5 : 1.0;
}

constexpr int RESID_NT = 256;

// The two neighbours of a point along one axis, for a fixed index i on that
// axis: neighbour = a * phi[idx + d] + b * phi[idx], which covers the
// interior (a = 1) and every closure of the boundary nodes (wrap-around or
// mirror offsets, Dirichlet zero a = b = 0, staggered Dirichlet b = -1,
// staggered Neumann b = 1; an axis without closure gives a zero difference).
struct Neighbours {
  int64_t dlo, dhi;
  double alo, ahi, blo, bhi;
};

// clo, chi: closures of the low and the high end of the axis.
__device__ __forceinline__ Neighbours neighbours(int64_t i, int64_t n, int64_t s, int clo, int chi) {
  Neighbours q{0, 0, 0.0, 0.0, 1.0, 1.0};
  if (clo == C_NONE) return q;
  if (i > 0) {
    q.dlo = -s; q.alo = 1.0; q.blo = 0.0;
  } else {
    switch (clo) {
      case C_PER: q.dlo = (n - 1) * s; q.alo = 1.0; q.blo = 0.0; break;
      case C_DV: q.blo = 0.0; break;
      case C_DS: q.blo = -1.0; break;
      case C_NV: q.dlo = s; q.alo = 1.0; q.blo = 0.0; break;
      default: break;  // C_NS: phi itself
    }
  }
  if (i < n - 1) {
    q.dhi = s; q.ahi = 1.0; q.bhi = 0.0;
  } else {
    switch (chi) {
      case C_PER: q.dhi = -(n - 1) * s; q.ahi = 1.0; q.bhi = 0.0; break;
      case C_DV: q.bhi = 0.0; break;
      case C_DS: q.bhi = -1.0; break;
      case C_NV: q.dhi = -s; q.ahi = 1.0; q.bhi = 0.0; break;
      default: break;
    }
  }
  return q;
}

// Second difference along axis 0 from values held in registers.
__device__ __forceinline__ double second_diff_reg(double lo_v, double c, double hi_v, int64_t i, int64_t n, int clo,
                                                  int chi, double lo_far, double hi_far) {
  if (clo == C_NONE) return 0.0;
  double lo, hi;
  if (i > 0) lo = lo_v;
  else {
    switch (clo) {
      case C_PER: lo = lo_far; break;   // phi[n-1]
      case C_DV: lo = 0.0; break;
      case C_DS: lo = -c; break;
      case C_NV: lo = hi_v; break;      // phi[1]
      default: lo = c; break;
    }
  }
  if (i < n - 1) hi = hi_v;
  else {
    switch (chi) {
      case C_PER: hi = hi_far; break;   // phi[0]
      case C_DV: hi = 0.0; break;
      case C_DS: hi = -c; break;
      case C_NV: hi = lo_v; break;      // phi[n-2]
      default: hi = c; break;
    }
  }
  return lo - 2.0 * c + hi;
}

// Block `blk` of `nblk` over one grid.  The work unit is a strip of RESID_NT
// consecutive points along axis 2, at a fixed axis-1 index, over a segment of
// RESID_SEG planes of axis 0.  The block marches the segment along axis 0 with
// the axis-0 neighbours in registers, so each value of phi comes from memory
// about once (plus one halo plane per segment); short segments give many
// independent workgroups to hide memory latency.
constexpr int RESID_SEG = 32;

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD
// b mod 8), each with its own L2.  Renumber them so that each XCD works on a
// contiguous range of units: the axis-1 neighbour rows a unit reads are then
// the rows of units on the same XCD, and come from its L2 instead of HBM.
// A bijection of [0, G).
__device__ __forceinline__ int64_t xcd_unit(int64_t b, int64_t G) {
  constexpr int64_t kXcd = 8;
  const int64_t q = G / kXcd, r = G % kXcd;
  const int64_t x = b % kXcd, i = b / kXcd;
  return x * q + (x < r ? x : r) + i;
}

// The same residual two points per thread along axis 2 (16-byte loads of
// phi and g, one 8-byte load for each end of the pair): fewer, wider
// requests for the same bytes.  Needs an even n2, unit strides along axis 2,
// even strides elsewhere and 16-byte aligned phi and g (checked by the
// caller).  A unit is a strip of 2 RESID_NT points; the blocks beyond the
// unit count stay idle.
__device__ __forceinline__ void resid_pairs(const ResidArgs& a, int64_t blk, int64_t nblk, double mg, double* s_wphi,
                                            double* s_wg, double* s_r2, double* s_g2) {
  const int64_t n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
  constexpr int W = 2 * RESID_NT;
  const int64_t strips = (n2 + W - 1) / W;
  const int64_t segs = (n0 + RESID_SEG - 1) / RESID_SEG;
  const int64_t units = strips * n1 * segs;
  const int64_t G = nblk < units ? nblk : units;
  if (blk >= G) return;
  const int64_t plane = n1 * n2;
  const double* __restrict__ phi = a.phi;
  const double* __restrict__ g = a.g;
  double* __restrict__ r64 = a.r && a.r_f64 ? static_cast<double*>(a.r) : nullptr;
  float* __restrict__ r32 = a.r && !a.r_f64 ? static_cast<float*>(a.r) : nullptr;
  for (int64_t u = xcd_unit(blk, G); u < units; u += G) {
    const int64_t seg = u / (strips * n1);
    const int64_t rem = u - seg * strips * n1;
    const int64_t i1 = rem / strips;
    const int64_t i2 = (rem - i1 * strips) * W + 2 * int64_t(threadIdx.x);
    if (i2 >= n2) continue;
    const int64_t p0 = a.ps[0], g0 = a.gs[0];
    const int64_t base = i1 * n2 + i2;
    const double w1 = axis_weight(a.clo[1], a.chi[1], i1, n1);
    const double wa = w1 * axis_weight(a.clo[2], a.chi[2], i2, n2);
    const double wb = w1 * axis_weight(a.clo[2], a.chi[2], i2 + 1, n2);
    // low end of point a and high end of point b (the pair's inner
    // neighbours are each other)
    const Neighbours qa = neighbours(i2, n2, 1, a.clo[2], a.chi[2]);
    const Neighbours qb = neighbours(i2 + 1, n2, 1, a.clo[2], a.chi[2]);
    const Neighbours q1 = neighbours(i1, n1, a.ps[1], a.clo[1], a.chi[1]);
    const double* __restrict__ pp = phi + i1 * a.ps[1] + i2;
    const double* __restrict__ gp = g + i1 * a.gs[1] + i2;
    auto ld2 = [](const double* q) { return *reinterpret_cast<const double2*>(q); };
    const double2 first = ld2(pp);
    const double2 last = ld2(pp + (n0 - 1) * p0);
    const int64_t s0 = seg * RESID_SEG;
    const int64_t s1 = (s0 + RESID_SEG < n0) ? s0 + RESID_SEG : n0;
    double2 prev = s0 > 0 ? ld2(pp + (s0 - 1) * p0) : double2{0.0, 0.0};
    double2 cur = ld2(pp + s0 * p0);
    double2 next = s0 + 1 < n0 ? ld2(pp + (s0 + 1) * p0) : cur;
    int64_t o = s0 * p0, og = s0 * g0, orr = s0 * plane;
#pragma unroll 2
    for (int64_t i0 = s0; i0 < s1; ++i0, o += p0, og += g0, orr += plane) {
      const double2 gv = ld2(gp + og);
      const double left = pp[o + qa.dlo], right = pp[o + 1 + qb.dhi];
      const double2 dn = ld2(pp + o + q1.dlo), up = ld2(pp + o + q1.dhi);
      const double d2a = qa.alo * left + qa.blo * cur.x - 2.0 * cur.x + cur.y;
      const double d2b = cur.x - 2.0 * cur.y + qb.ahi * right + qb.bhi * cur.y;
      const double d1a = q1.alo * dn.x + q1.blo * cur.x - 2.0 * cur.x + q1.ahi * up.x + q1.bhi * cur.x;
      const double d1b = q1.alo * dn.y + q1.blo * cur.y - 2.0 * cur.y + q1.ahi * up.y + q1.bhi * cur.y;
      const double d0a = second_diff_reg(prev.x, cur.x, next.x, i0, n0, a.clo[0], a.chi[0], last.x, first.x);
      const double d0b = second_diff_reg(prev.y, cur.y, next.y, i0, n0, a.clo[0], a.chi[0], last.y, first.y);
      const double la = a.inv_h2[2] * d2a + a.inv_h2[1] * d1a + a.inv_h2[0] * d0a - a.shift * cur.x;
      const double lb = a.inv_h2[2] * d2b + a.inv_h2[1] * d1b + a.inv_h2[0] * d0b - a.shift * cur.y;
      const double gca = gv.x - mg, gcb = gv.y - mg;
      const double ra = gca - la, rb = gcb - lb;
      if (r64) *reinterpret_cast<double2*>(r64 + base + orr) = double2{ra, rb};
      else if (r32) *reinterpret_cast<float2*>(r32 + base + orr) = float2{float(ra), float(rb)};
      const double w0 = axis_weight(a.clo[0], a.chi[0], i0, n0);
      *s_wphi += w0 * (wa * cur.x + wb * cur.y);
      *s_wg += w0 * (wa * gv.x + wb * gv.y);
      *s_r2 += ra * ra + rb * rb;
      *s_g2 += gca * gca + gcb * gcb;
      prev = cur;
      cur = next;
      next = (i0 + 2 < n0) ? ld2(pp + o + 2 * p0) : cur;
    }
  }
}

// Whether the two-point path applies (uniform for the launch).
__device__ __forceinline__ bool resid_pairs_ok(const ResidArgs& a) {
  const uintptr_t al = reinterpret_cast<uintptr_t>(a.phi) | reinterpret_cast<uintptr_t>(a.g) |
                       (a.r ? reinterpret_cast<uintptr_t>(a.r) : 0);
  return a.phi && a.n[2] >= 2 && a.n[2] % 2 == 0 && a.ps[2] == 1 && a.gs[2] == 1 &&
         ((a.ps[0] | a.ps[1] | a.gs[0] | a.gs[1]) & 1) == 0 && (al & 15) == 0;
}

__device__ __forceinline__ void resid_body(const ResidArgs& a, int64_t blk, int64_t nblk, double* part) {
  const int64_t n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
  const int64_t strips = (n2 + RESID_NT - 1) / RESID_NT;
  const int64_t segs = (n0 + RESID_SEG - 1) / RESID_SEG;
  const int64_t units = strips * n1 * segs;
  const int64_t plane = n1 * n2;
  const double mg = a.mg ? a.mg[0] : 0.0;
  double s_wphi = 0.0, s_wg = 0.0, s_r2 = 0.0, s_g2 = 0.0;
  if (!a.phi) {
    // sums of g alone (weighted mean of the right-hand side): one read of g
    for (int64_t u = xcd_unit(blk, nblk); u < units; u += nblk) {
      const int64_t seg = u / (strips * n1);
      const int64_t rem = u - seg * strips * n1;
      const int64_t i1 = rem / strips;
      const int64_t i2 = (rem - i1 * strips) * RESID_NT + threadIdx.x;
      if (i2 >= n2) continue;
      const int64_t gbase = i1 * a.gs[1] + i2 * a.gs[2];
      const double w12 = axis_weight(a.clo[1], a.chi[1], i1, n1) * axis_weight(a.clo[2], a.chi[2], i2, n2);
      const int64_t s0 = seg * RESID_SEG;
      const int64_t s1 = (s0 + RESID_SEG < n0) ? s0 + RESID_SEG : n0;
#pragma unroll 4
      for (int64_t i0 = s0; i0 < s1; ++i0) {
        const double gv = a.g[i0 * a.gs[0] + gbase];
        const double gc = gv - mg;
        s_wg += w12 * axis_weight(a.clo[0], a.chi[0], i0, n0) * gv;
        s_g2 += gc * gc;
      }
    }
  }
  const bool pairs = resid_pairs_ok(a);
  if (pairs) resid_pairs(a, blk, nblk, mg, &s_wphi, &s_wg, &s_r2, &s_g2);
  // distinct arrays: the loads of later planes may move above the stores of r
  const double* __restrict__ phi = pairs ? nullptr : a.phi;
  const double* __restrict__ g = a.g;
  double* __restrict__ r64 = a.r && a.r_f64 ? static_cast<double*>(a.r) : nullptr;
  float* __restrict__ r32 = a.r && !a.r_f64 ? static_cast<float*>(a.r) : nullptr;
  for (int64_t u = xcd_unit(blk, nblk); phi && u < units; u += nblk) {
    const int64_t seg = u / (strips * n1);
    const int64_t rem = u - seg * strips * n1;
    const int64_t i1 = rem / strips;
    const int64_t i2 = (rem - i1 * strips) * RESID_NT + threadIdx.x;
    if (i2 >= n2) continue;
    // phi and g may be views into larger (halo-padded) arrays: their own
    // strides; r is C-contiguous
    const int64_t p0 = a.ps[0], g0 = a.gs[0];
    const int64_t base = i1 * n2 + i2;
    const double w12 = axis_weight(a.clo[1], a.chi[1], i1, n1) * axis_weight(a.clo[2], a.chi[2], i2, n2);
    // axes 2 and 1: neighbour offsets and weights are fixed for this thread
    const Neighbours q2 = neighbours(i2, n2, a.ps[2], a.clo[2], a.chi[2]);
    const Neighbours q1 = neighbours(i1, n1, a.ps[1], a.clo[1], a.chi[1]);
    const double* __restrict__ pp = phi + i1 * a.ps[1] + i2 * a.ps[2];
    const double* __restrict__ gp = g + i1 * a.gs[1] + i2 * a.gs[2];
    const double first = pp[0];
    const double last = pp[(n0 - 1) * p0];
    const int64_t s0 = seg * RESID_SEG;
    const int64_t s1 = (s0 + RESID_SEG < n0) ? s0 + RESID_SEG : n0;
    double prev = s0 > 0 ? pp[(s0 - 1) * p0] : 0.0;
    double cur = pp[s0 * p0];
    double next = s0 + 1 < n0 ? pp[(s0 + 1) * p0] : cur;
    int64_t o = s0 * p0, og = s0 * g0, orr = s0 * plane;
#pragma unroll 4
    for (int64_t i0 = s0; i0 < s1; ++i0, o += p0, og += g0, orr += plane) {
      const double gv = gp[og];
      const double d2 = q2.alo * pp[o + q2.dlo] + q2.blo * cur - 2.0 * cur + q2.ahi * pp[o + q2.dhi] + q2.bhi * cur;
      const double d1 = q1.alo * pp[o + q1.dlo] + q1.blo * cur - 2.0 * cur + q1.ahi * pp[o + q1.dhi] + q1.bhi * cur;
      const double lap = a.inv_h2[2] * d2 + a.inv_h2[1] * d1 +
                         a.inv_h2[0] * second_diff_reg(prev, cur, next, i0, n0, a.clo[0], a.chi[0], last, first) -
                         a.shift * cur;
      const double gc = gv - mg;
      const double r = gc - lap;
      if (r64) r64[base + orr] = r;
      else if (r32) r32[base + orr] = float(r);
      const double w = w12 * axis_weight(a.clo[0], a.chi[0], i0, n0);
      s_wphi += w * cur;
      s_wg += w * gv;
      s_r2 += r * r;
      s_g2 += gc * gc;
      prev = cur;
      cur = next;
      next = (i0 + 2 < n0) ? pp[o + 2 * p0] : cur;
    }
  }
  __shared__ double red[4][RESID_NT];
  red[0][threadIdx.x] = s_wphi;
  red[1][threadIdx.x] = s_wg;
  red[2][threadIdx.x] = s_r2;
  red[3][threadIdx.x] = s_g2;
  __syncthreads();
  for (int off = RESID_NT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(RESID_NT) resid_kernel(ResidArgs a) {
  resid_body(a, blockIdx.x, gridDim.x, a.partials + int64_t(blockIdx.x) * 4);
}

__global__ void __launch_bounds__(RESID_NT) resid_batch_kernel(BatchResidArgs b) {
  const int pi = b.blk_prob[blockIdx.x];
  ResidArgs a = b.args[pi];
  a.phi = b.phi_tab ? static_cast<const double*>(b.phi_tab[pi]) : nullptr;
  a.g = static_cast<const double*>(b.g_tab[pi]);
  a.r = b.r_tab ? b.r_tab[pi] : nullptr;
  a.r_f64 = b.r_f64;
  a.mg = (b.use_mg && a.singular) ? b.scalars + int64_t(pi) * S_COUNT + S_MG : nullptr;
  const int blk = int(blockIdx.x) - b.blk_start[pi];
  resid_body(a, blk, b.blk_count[pi], b.partials + int64_t(blockIdx.x) * 4);
}

// Sum block partials [first, first + count) in a fixed order and derive the
// gauge shift and the weighted mean of g.
__device__ __forceinline__ void finalize_body(const double* __restrict__ partials, int first, int count,
                                              double inv_wsum, double* __restrict__ scalars) {
  __shared__ double red[4][256];
  double s[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < count; b += 256)
    for (int q = 0; q < 4; ++q) s[q] += partials[int64_t(first + b) * 4 + q];
  for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    scalars[S_WPHI] = red[0][0];
    scalars[S_WG] = red[1][0];
    scalars[S_R2] = red[2][0];
    scalars[S_G2] = red[3][0];
    scalars[S_SHIFT] = red[0][0] * inv_wsum;
    scalars[S_MG] = red[1][0] * inv_wsum;
  }
}

__global__ void __launch_bounds__(256) finalize_kernel(const double* __restrict__ partials, int nblocks,
                                                       double inv_wsum, double* __restrict__ scalars) {
  finalize_body(partials, 0, nblocks, inv_wsum, scalars);
}

// One block per grid.
__global__ void __launch_bounds__(256) finalize_batch_kernel(const double* __restrict__ partials,
                                                             const int* __restrict__ blk_start,
                                                             const int* __restrict__ blk_count,
                                                             const double* __restrict__ inv_wsum,
                                                             double* __restrict__ scalars) {
  const int pi = blockIdx.x;
  finalize_body(partials, blk_start[pi], blk_count[pi], inv_wsum[pi], scalars + int64_t(pi) * S_COUNT);
}

// Fill a double array with zeros (used instead of memset nodes so the sequence is graph-safe).
__global__ void zero_kernel(double* p, int64_t count) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}


// Blocks of one residual launch: one per (axis-1 index, strip of axis 2,
// segment of axis 0), at most 16384.
int resid_blocks(const int64_t n[3]) {
  const int64_t units =
      n[1] * ((n[2] + RESID_NT - 1) / RESID_NT) * ((n[0] + RESID_SEG - 1) / RESID_SEG);
  return int(units < 16384 ? units : 16384);
}

hipError_t launch_resid(const ResidArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(resid_kernel, dim3(resid_blocks(a.n)), dim3(RESID_NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int nblocks, double inv_wsum, double* scalars, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, partials, nblocks, inv_wsum, scalars);
  return hipGetLastError();
}

hipError_t launch_resid_batch(const BatchResidArgs& b, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(resid_batch_kernel, dim3(blocks), dim3(RESID_NT), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_finalize_batch(const double* partials, const int* blk_start, const int* blk_count,
                                 const double* inv_wsum, double* scalars, int count, hipStream_t s) {
  hipLaunchKernelGGL(finalize_batch_kernel, dim3(count), dim3(256), 0, s, partials, blk_start, blk_count, inv_wsum,
                     scalars);
  return hipGetLastError();
}

hipError_t launch_zero(double* p, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(zero_kernel, dim3(64), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

}  // namespace mpois
