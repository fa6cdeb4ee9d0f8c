// Two axes of a small grid in one sweep: a workgroup holds a whole plane of
// the last two axes (n x n values, fixed index along axis 0) in LDS and runs
// the line transforms of both axes on it, with an LDS transpose between them.
// A 3D solve then takes three launches (forward planes, the fused axis-0
// sweep, inverse planes) instead of five; for grids this small (32^3) the
// launches, not the bytes, set the time.  The transforms are those of the
// line passes (pack / DFT / unpack of transform_phase), compiled for one
// length, the same on both axes.
#pragma once

#include "line_pass.h"

namespace mpois {

// Forward (INV false): read the plane, transform along axis 2 (rows as
// lines), transpose, transform along axis 1 (columns as lines), write.
// Inverse: the same with axis 1 first.  a2 / a1 describe the passes along the
// last / middle axis (tables, kinds); the source (and its element type) is
// the first pass's, the destination (type, update mode) the second's.  Both
// arrays are C-contiguous; plane b starts at element b * N * N.
// Stage twiddles of a compile-time stage list: ns (R - 1) per stage, ns the
// product of the radices before it.
template <int... Rs>
constexpr int stage_twiddles() {
  int ns = 1, total = 0;
  for (int r : {Rs...}) {
    total += ns * (r - 1);
    ns *= r;
  }
  return total;
}

template <bool INV, typename T, int NT, int N, int M, int P, int KF, int KB, int... Rs>
__global__ void __launch_bounds__(NT) plane_pass(PassArgs a2, PassArgs a1) {
  constexpr int K = INV ? KB : KF;  // kind of both phases
  constexpr int NP = N / 2;  // a tile of N lines: N / 2 pairs
  constexpr int ZP = NP;
  constexpr int XP = 2 * ZP;
  constexpr int NN = N * N;
  constexpr int E = (NN + NT - 1) / NT;
  static_assert(N % 2 == 0 && NT % N == 0, "plane tiles need an even n that divides the thread count");
  using AX = Ax<N, M, P>;
  using ST = StageList<Rs...>;
  extern __shared__ __align__(16) unsigned char smem[];
  T* X = reinterpret_cast<T*>(smem);
  cx<T>* Z = reinterpret_cast<cx<T>*>(smem);
  const PassArgs& first = INV ? a1 : a2;
  const PassArgs& second = INV ? a2 : a1;
  const int64_t base = int64_t(blockIdx.x) * NN;
  const int tid = int(threadIdx.x);

  // element (i1, i2) of the plane: lines are rows (i1) when axis 2 goes
  // first, columns (i2) when axis 1 does
  auto load = [&](auto elem) {
    using S = decltype(elem);
    const S* src = static_cast<const S*>(first.src) + base;
    S v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int e = tid + i * NT;
      v[i] = src[e < NN ? e : 0];
    }
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int e = tid + i * NT;
      if (e < NN) {
        const int i1 = e / N, i2 = e % N;
        X[INV ? i1 * XP + i2 : i2 * XP + i1] = T(v[i]);
      }
    }
  };
  if (first.src_f64) load(double(0));
  else load(float(0));
  // both axes use the same transform tables: their stage twiddles go to LDS
  // behind the plane, so that no stage waits on a global-memory read
  constexpr int NTW = stage_twiddles<Rs...>();
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem + spec_main_lds<T, N, P, ZP>());
  {
    const cx<T>* g = static_cast<const cx<T>*>(first.ax.tw);
    for (int i = tid; i < NTW; i += NT) tw[i] = g[i];
  }
  AxisDev d1 = first.ax, d2 = second.ax;
  d1.tw = tw;
  d2.tw = tw;
  __syncthreads();

  bool mirrored = false;
  transform_phase<T, NP, NT, P, 0, 0, AX, ST, K, ZP>(X, Z, AX{d1}, first, 0, K, false, -1, mirrored);

  // transpose: value of line t, element j moves from X[j * XP + t] to X[t * XP + j]
  {
    T v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int e = tid + i * NT;
      if (e < NN) v[i] = X[(e % N) * XP + e / N];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int e = tid + i * NT;
      if (e < NN) X[(e / N) * XP + e % N] = v[i];
    }
    __syncthreads();
  }
  mirrored = false;
  transform_phase<T, NP, NT, P, 0, 0, AX, ST, K, ZP>(X, Z, AX{d2}, second, 0, K, false, -1, mirrored);

  // store element (i1, i2): after the second phase the lines are columns
  // (forward) or rows (inverse)
  const double shift = (second.update && second.shift) ? second.shift[0] : 0.0;
  auto store = [&](auto elem, bool update) {
    using D = decltype(elem);
    D* dst = static_cast<D*>(second.dst) + base;
    T v[E];
    D old[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int e = tid + i * NT;
      if (e < NN) {
        const int i1 = e / N, i2 = e % N;
        v[i] = X[INV ? i2 * XP + i1 : i1 * XP + i2];
        if (update) old[i] = dst[e];
      }
    }
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int e = tid + i * NT;
      if (e < NN) dst[e] = update ? D(double(old[i]) + double(v[i]) - shift) : D(v[i]);
    }
  };
  if (second.update) store(double(0), true);
  else if (second.dst_f64) store(double(0), false);
  else store(float(0), false);
}

template <typename T, int NT, int N, int M, int P, int KF, int KB, int... Rs>
constexpr int plane_lds() {
  return spec_main_lds<T, N, P, N / 2>() + stage_twiddles<Rs...>() * 2 * int(sizeof(T));
}

template <typename T, int NT, int N, int M, int P, int KF, int KB, int... Rs>
hipError_t launch_plane_t(const PassArgs& a2, const PassArgs& a1, int inverse, int64_t planes, hipStream_t s) {
  const int k = inverse ? KB : KF;
  for (const PassArgs* a : {&a2, &a1})
    if (a->ax.n != N || a->ax.M != M || a->ax.P != P || a->ax.nstages != int(sizeof...(Rs)) || a->kind_f != k ||
        a->kind_b != -1)
      return hipErrorInvalidValue;  // both axes must be the transform this kernel was compiled for
  if (a2.ax.tw != a1.ax.tw) return hipErrorInvalidValue;  // one twiddle table serves both
  constexpr int lds = plane_lds<T, NT, N, M, P, KF, KB, Rs...>();
  if (inverse)
    hipLaunchKernelGGL((plane_pass<true, T, NT, N, M, P, KF, KB, Rs...>), dim3(unsigned(planes)), dim3(NT), lds, s,
                       a2, a1);
  else
    hipLaunchKernelGGL((plane_pass<false, T, NT, N, M, P, KF, KB, Rs...>), dim3(unsigned(planes)), dim3(NT), lds, s,
                       a2, a1);
  return hipGetLastError();
}

}  // namespace mpois
