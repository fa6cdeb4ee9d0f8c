// Line-transform kernel of the fast Poisson solver for gfx950 (CDNA4).
//
// line_pass: one HBM sweep along one axis.  A workgroup owns a tile of TL = 2*NP
// adjacent lines: it loads them into LDS with the lines innermost (TL-wide
// segments of the TL lines per request), packs two real lines into one
// complex sequence per pair (in place for the DCT-I and the real DFT, whose
// packed layout is the tile layout itself), runs a Stockham DFT over all
// pairs at once in LDS (or a Bluestein chirp convolution when the length has a
// prime factor the codelets do not cover), unpacks, and stores.  The same
// sweep can also apply the eigenvalue division and the inverse transform of
// the axis, so the middle of a solve costs one sweep instead of two.
//
// The transforms are those of Table 2 of the paper (DFT for periodic axes,
// DST-I/II for Dirichlet, DCT-I/II for Neumann, with DST-III/DCT-III as the
// staggered-grid inverses); periodic axes use the real half-complex form of
// the DFT so every sweep is real-to-real and in place.  The divisor is the sum
// of the per-axis eigenvalues (Section 2.3), from Table 3 or Table 4.
#pragma once
#include <hip/hip_runtime.h>


#include "internal.h"

namespace mpois {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
// multiply by -i
template <typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.im, -a.re}; }
// c ? a : b per component (a conditional on the struct itself would select
// between addresses and keep the operands in scratch memory)
template <typename T>
__device__ __forceinline__ cx<T> csel(bool c, cx<T> a, cx<T> b) { return {c ? a.re : b.re, c ? a.im : b.im}; }

// x / d from the hardware reciprocal and Newton steps (two in FP64, one in
// FP32) and a final correction of the quotient: within an ulp or so of the
// rounded quotient, at a fraction of the cost of IEEE division.  Used by the
// specialised kernels for the eigenvalue division.
__device__ __forceinline__ float quick_div(float x, float d) {
  float r = __builtin_amdgcn_rcpf(d);
  r = __builtin_fmaf(__builtin_fmaf(-d, r, 1.0f), r, r);
  const float q = x * r;
  return __builtin_fmaf(__builtin_fmaf(-d, q, x), r, q);
}
__device__ __forceinline__ double quick_div(double x, double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
  r = __builtin_fma(__builtin_fma(-d, r, 1.0), r, r);
  const double q = x * r;
  return __builtin_fma(__builtin_fma(-d, q, x), r, q);
}

// Length view of one axis transform.  Ax<> reads the line length n, the
// complex DFT length M and the work length P (P > M: Bluestein) from the
// device description at run time; Ax<N, M, P> makes them compile-time
// constants, so a kernel specialised for one length folds its index
// arithmetic and sizes its loops exactly.  Table pointers always come from
// the description.
template <int N_ = 0, int M_ = 0, int P_ = 0>
struct Ax {
  const AxisDev& d;
  static constexpr bool ct = N_ != 0;
  static constexpr int Nc = N_, Mc = M_, Pc = P_;
  __device__ __forceinline__ int n() const {
    if constexpr (ct) return N_; else return d.n;
  }
  __device__ __forceinline__ int M() const {
    if constexpr (ct) return M_; else return d.M;
  }
  __device__ __forceinline__ int P() const {
    if constexpr (ct) return P_; else return d.P;
  }
  __device__ __forceinline__ bool blue() const {
    if constexpr (ct) return P_ != M_; else return d.bluestein != 0;
  }
};

// Thread index hidden from loop-invariant code motion: per-item address
// arithmetic is then recomputed where it is used instead of being hoisted out
// of the phase / stage loops and kept live (which spills).
__device__ __forceinline__ int opaque_tid() {
  int t = int(threadIdx.x);
  asm volatile("" : "+v"(t));
  return t;
}

// ----------------------------------------------------------------------------- compile-time trig
// cos / sin of 2 pi k / n evaluated by the compiler: reduce to [0, pi/4] by the
// quadrant and octant symmetries, then sum the Taylor series (enough terms for
// double precision on that interval).
constexpr double kTwoPi = 6.283185307179586476925286766559005768;
constexpr double ct_sin_series(double x) {
  double term = x, sum = x;
  for (int i = 1; i < 14; ++i) {
    term *= -x * x / double((2 * i) * (2 * i + 1));
    sum += term;
  }
  return sum;
}
constexpr double ct_cos_series(double x) {
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < 14; ++i) {
    term *= -x * x / double((2 * i - 1) * (2 * i));
    sum += term;
  }
  return sum;
}
// (cos, sin)(2 pi k / n) for integers; 8k/n selects the octant exactly.
constexpr double ct_cs(long k, long n, bool want_sin) {
  long r = ((k % n) + n) % n;
  long oct = (8 * r) / n;             // 0..7
  // angle within the octant, measured from the octant's start or end
  double t = kTwoPi * double(8 * r - oct * n) / double(8 * n);  // in [0, pi/4)
  double c = 0, s = 0;
  switch (oct) {
    case 0: c = ct_cos_series(t); s = ct_sin_series(t); break;
    case 1: { double u = kTwoPi / 8 - t; c = ct_sin_series(u); s = ct_cos_series(u); break; }
    case 2: c = -ct_sin_series(t); s = ct_cos_series(t); break;
    case 3: { double u = kTwoPi / 8 - t; c = -ct_cos_series(u); s = ct_sin_series(u); break; }
    case 4: c = -ct_cos_series(t); s = -ct_sin_series(t); break;
    case 5: { double u = kTwoPi / 8 - t; c = -ct_sin_series(u); s = -ct_cos_series(u); break; }
    case 6: c = ct_sin_series(t); s = -ct_cos_series(t); break;
    default: { double u = kTwoPi / 8 - t; c = ct_cos_series(u); s = -ct_sin_series(u); break; }
  }
  return want_sin ? s : c;
}
constexpr double ct_cos(long k, long n) { return ct_cs(k, n, false); }
constexpr double ct_sin(long k, long n) { return ct_cs(k, n, true); }

// Table of (cos, sin)(2 pi k / N), k < N, built by the compiler.
template <int N>
struct TwTable {
  double c[N];
  double s[N];
  constexpr TwTable() : c(), s() {
    for (int k = 0; k < N; ++k) {
      c[k] = ct_cos(k, N);
      s[k] = ct_sin(k, N);
    }
  }
};
template <int N>
struct Tw {
  static constexpr TwTable<N> t{};
};

// Modular arithmetic for the Rader permutation (compile time).
constexpr long ct_powmod(long b, long e, long m) {
  long r = 1;
  b %= m;
  while (e > 0) {
    if (e & 1) r = r * b % m;
    b = b * b % m;
    e >>= 1;
  }
  return r;
}
// Smallest primitive root of a prime p (declared below the tables that use it).
constexpr long ct_primroot(long p);

constexpr long ct_primroot(long p) {
  for (long g = 2; g < p; ++g) {
    bool ok = true;
    for (long q = 2; q <= p - 1 && ok; ++q) {
      bool prime = true;
      for (long d = 2; d * d <= q; ++d)
        if (q % d == 0) prime = false;
      if (prime && (p - 1) % q == 0 && ct_powmod(g, (p - 1) / q, p) == 1) ok = false;
    }
    if (ok) return g;
  }
  return 0;
}


// ----------------------------------------------------------------------------- codelets
// Forward DFT (kernel e^{-2 pi i jk/R}) of R values held in registers.

template <typename T>
__device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename T>
__device__ __forceinline__ void dft4(cx<T>* v) {
  cx<T> t0 = v[0] + v[2], t1 = v[0] - v[2], t2 = v[1] + v[3], t3 = mul_mi(v[1] - v[3]);
  v[0] = t0 + t2;
  v[2] = t0 - t2;
  v[1] = t1 + t3;
  v[3] = t1 - t3;
}

template <typename T>
__device__ __forceinline__ void dft8(cx<T>* v) {
  const T r2 = T(0.70710678118654752440084436210484903928483593768847);
  cx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4(e);
  dft4(o);
  // twiddles e^{-2 pi i k/8}, k = 0..3
  cx<T> o1 = {(o[1].re + o[1].im) * r2, (o[1].im - o[1].re) * r2};
  cx<T> o2 = mul_mi(o[2]);
  cx<T> o3 = {(o[3].im - o[3].re) * r2, -(o[3].re + o[3].im) * r2};
  v[0] = e[0] + o[0];
  v[4] = e[0] - o[0];
  v[1] = e[1] + o1;
  v[5] = e[1] - o1;
  v[2] = e[2] + o2;
  v[6] = e[2] - o2;
  v[3] = e[3] + o3;
  v[7] = e[3] - o3;
}

template <typename T>
__device__ __forceinline__ void dft3(cx<T>* v) {
  const T s1 = T(0.86602540378443864676372317075293618347140262690519);
  cx<T> t = v[1] + v[2], d = v[1] - v[2];
  cx<T> m = {v[0].re - T(0.5) * t.re, v[0].im - T(0.5) * t.im};
  v[0] = v[0] + t;
  v[1] = {m.re + s1 * d.im, m.im - s1 * d.re};
  v[2] = {m.re - s1 * d.im, m.im + s1 * d.re};
}

// Odd radix R >= 5 from the symmetric form: with s_j = v_j + v_{R-j} and
// d_j = v_j - v_{R-j},  X_k = v_0 + sum_j s_j cos(2 pi jk/R) - i sum_j d_j sin(2 pi jk/R)
// and X_{R-k} is the same with +i.
template <typename T, int R>
__device__ __forceinline__ void dft_odd(cx<T>* v) {
  constexpr int H = (R - 1) / 2;
  cx<T> s[H], d[H];
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    s[j - 1] = v[j] + v[R - j];
    d[j - 1] = v[j] - v[R - j];
  }
  cx<T> a0 = v[0];
  cx<T> x0 = a0;
#pragma unroll
  for (int j = 0; j < H; ++j) x0 = x0 + s[j];
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    cx<T> A = a0, B = {T(0), T(0)};
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const T c = T(Tw<R>::t.c[(j * k) % R]);
      const T sn = T(Tw<R>::t.s[(j * k) % R]);
      A.re += s[j - 1].re * c;
      A.im += s[j - 1].im * c;
      B.re += d[j - 1].re * sn;
      B.im += d[j - 1].im * sn;
    }
    v[k] = {A.re + B.im, A.im - B.re};
    v[R - k] = {A.re - B.im, A.im + B.re};
  }
  v[0] = x0;
}

template <typename T, int R>
__device__ __forceinline__ void dft_any(cx<T>* v);

// Two-level codelet for R = R1 * R2: DFT-R1 over each stride-R2 subsequence,
// twiddle e^{-2 pi i j2 k1 / R}, DFT-R2 across subsequences, output k1 + R1 k2.
template <typename T, int R1, int R2>
__device__ __forceinline__ void dft_2level(cx<T>* v) {
  constexpr int R = R1 * R2;
  cx<T> t[R2][R1];
#pragma unroll
  for (int j2 = 0; j2 < R2; ++j2) {
#pragma unroll
    for (int j1 = 0; j1 < R1; ++j1) t[j2][j1] = v[j1 * R2 + j2];
    dft_any<T, R1>(t[j2]);
#pragma unroll
    for (int k1 = 1; k1 < R1; ++k1) {
      if (j2 == 0) continue;
      const cx<T> w = {T(Tw<R>::t.c[j2 * k1]), T(-Tw<R>::t.s[j2 * k1])};
      t[j2][k1] = cmul(t[j2][k1], w);
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cx<T> u[R2];
#pragma unroll
    for (int j2 = 0; j2 < R2; ++j2) u[j2] = t[j2][k1];
    dft_any<T, R2>(u);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = u[k2];
  }
}

// Prime-factor (Good-Thomas) codelet for coprime R1, R2: input n = (R2 n1 +
// R1 n2) mod R, DFT-R1 over n1, DFT-R2 over n2, output k with k = k1 mod R1
// and k = k2 mod R2 (Chinese remainder map); no twiddle factors.
constexpr int ct_modinv(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;
}

template <typename T, int R1, int R2>
__device__ __forceinline__ void dft_pfa(cx<T>* v) {
  constexpr int R = R1 * R2;
  constexpr int e1 = R2 * ct_modinv(R2 % R1, R1);  // = 1 mod R1, 0 mod R2
  constexpr int e2 = R1 * ct_modinv(R1 % R2, R2);  // = 0 mod R1, 1 mod R2
  cx<T> t[R2][R1];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) t[n2][n1] = v[(R2 * n1 + R1 * n2) % R];
    dft_any<T, R1>(t[n2]);
  }
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cx<T> u[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) u[n2] = t[n2][k1];
    dft_any<T, R2>(u);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[(e1 * k1 + e2 * k2) % R] = u[k2];
  }
}

template <typename T, int R>
__device__ __forceinline__ void dft_any(cx<T>* v) {
  if constexpr (R == 1) return;
  else if constexpr (R == 2) dft2(v);
  else if constexpr (R == 3) dft3(v);
  else if constexpr (R == 4) dft4(v);
  else if constexpr (R == 8) dft8(v);
  else if constexpr (R == 9) dft_2level<T, 3, 3>(v);
  else if constexpr (R == 14) dft_pfa<T, 7, 2>(v);
  else if constexpr (R == 16) dft_2level<T, 4, 4>(v);
  else if constexpr (R == 18) dft_pfa<T, 2, 9>(v);
  else if constexpr (R == 36) dft_pfa<T, 4, 9>(v);
  else if constexpr (R == 32) dft_2level<T, 8, 4>(v);
  else if constexpr (R == 64) dft_2level<T, 8, 8>(v);
  else if constexpr (R == 72) dft_pfa<T, 8, 9>(v);
  else dft_odd<T, R>(v);
}

// ----------------------------------------------------------------------------- Stockham stage
// Work buffer layout: Z[m * ZP + p] holds element m of pair p (ZP >= NP: the
// row pitch in complex values; a pitch above NP staggers the rows over the
// LDS banks).  All butterflies
// of the stage are read into registers before the barrier and written after
// it, so the stage runs in place in one buffer.
// PC, NSC: compile-time work length and stage stride (0: the run-time P, ns).
template <typename T, int R, int NP, int NT, int PMAX, int PC = 0, int NSC = 0, int ZP = NP>
__device__ __forceinline__ void stage(cx<T>* Z, int P_rt, int ns_rt, const cx<T>* __restrict__ tw,
                                      unsigned ns_mul = 0) {
  constexpr int NB = (((PC ? PC : PMAX) / R) * NP + NT - 1) / NT;
  const int P = PC ? PC : P_rt;
  const int ns = NSC ? NSC : ns_rt;
  const int nbp = P / R;      // butterflies per pair
  const int items = nbp * NP;
  const int tid = opaque_tid();
  // b mod ns: a constant, or (FP32 run-time stage lists; b < 2^16) a
  // multiply by the stage's scaled reciprocal.  The FP64 shapes held to 128
  // registers keep the division: the reciprocal's registers made them spill.
  auto mod_ns = [&](int b) -> int {
    if constexpr (NSC != 0) {
      return b % NSC;
    } else if constexpr (sizeof(T) == 4) {
      if (ns_mul) return b - int(__umulhi(unsigned(b), ns_mul)) * ns;
      return 0;  // ns == 1
    } else {
      return b % ns;
    }
  };
  cx<T> v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int item = tid + i * NT;
    if (item < items) {
      const int p = item % NP;
      const int b = item / NP;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = Z[(b + r * nbp) * ZP + p];
      if (ns > 1) {
        const int k = mod_ns(b);
        const cx<T>* w = tw + k * (R - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], w[r - 1]);
      }
      dft_any<T, R>(v[i]);
    }
  }
  __syncthreads();
  const int tid2 = opaque_tid();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int item = tid2 + i * NT;
    if (item < items) {
      const int p = item % NP;
      const int b = item / NP;
      const int k = mod_ns(b);
      const int base = (b - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) Z[(base + r * ns) * ZP + p] = v[i][r];
    }
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------- lane-parallel Rader
// Exchange of a value with lane (lane ^ mask), mask in {1, 2, 4}, through DPP
// lane moves (no LDS traffic): quad permutations for 1 and 2, and for 4 the
// mirror inside each group of 8 lanes (lane ^ 7) followed by lane ^ 3.
template <int MASK>
__device__ __forceinline__ int lane_xor_i32(int v) {
  static_assert(MASK == 1 || MASK == 2 || MASK == 4, "lane mask");
  if constexpr (MASK == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);  // [1,0,3,2]
  else if constexpr (MASK == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);  // [2,3,0,1]
  else {
    const int m = __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);  // half-row mirror
    return __builtin_amdgcn_update_dpp(0, m, 0x1B, 0xF, 0xF, true);           // [3,2,1,0]
  }
}

template <int MASK>
__device__ __forceinline__ float lane_xor(float v) {
  return __int_as_float(lane_xor_i32<MASK>(__float_as_int(v)));
}

template <int MASK>
__device__ __forceinline__ double lane_xor(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_xor_i32<MASK>(int(b & 0xffffffffLL));
  const int hi = lane_xor_i32<MASK>(int(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

template <int MASK, typename T>
__device__ __forceinline__ cx<T> lane_xor_cx(cx<T> v) {
  return {lane_xor<MASK>(v.re), lane_xor<MASK>(v.im)};
}

// e^{-2 pi i j / (2h)} for j < h <= 4.
template <typename T>
__device__ __forceinline__ cx<T> w2h(int j, int h) {
  const T r2 = T(0.70710678118654752440084436210484903928483593768847);
  if (h == 1 || j == 0) return {T(1), T(0)};
  if (h == 2 || j == 2) return {T(0), T(-1)};
  return {j == 1 ? r2 : -r2, -r2};
}

// One radix-2 step of a DFT of length G spread over G lanes (one value per
// lane, K independent columns), partner lane s ^ H, w = e^{-2 pi i (s mod H)/(2H)}.
// DIF (DIT=false): top lane x + x', bottom lane (x' - x) w.
// DIT (DIT=true):  top lane x + w x', bottom lane x' - w x.
// Both are written without per-value selects: with weff = 1 on the top lane
// and w on the bottom one, DIF is (x' + sg x) weff and DIT exchanges
// z = x weff and forms z' + sg z (sg = +1 top, -1 bottom).
template <typename T, int K, int H, bool DIT>
__device__ __forceinline__ void lane_radix2(cx<T>* x, int s) {
  const bool top = (s & H) == 0;
  const T sg = top ? T(1) : T(-1);
  const cx<T> weff = csel(top, cx<T>{T(1), T(0)}, w2h<T>(s & (H - 1), H));
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if constexpr (!DIT) {
      const cx<T> xp = lane_xor_cx<H>(x[k]);
      const cx<T> t = {xp.re + sg * x[k].re, xp.im + sg * x[k].im};
      x[k] = (H == 1) ? t : cmul(t, weff);
    } else {
      const cx<T> z = (H == 1) ? x[k] : cmul(x[k], weff);
      const cx<T> zp = lane_xor_cx<H>(z);
      x[k] = {zp.re + sg * z.re, zp.im + sg * z.im};
    }
  }
}

template <int G>
__device__ __forceinline__ int lane_bitrev(int s) {
  if constexpr (G == 2) return s;
  else if constexpr (G == 4) return ((s & 1) << 1) | (s >> 1);
  else return ((s & 1) << 2) | (s & 2) | ((s & 4) >> 2);
}

// Prime radix R by Rader's algorithm: with a primitive root g of R, the
// non-zero outputs are X[g^{-m}] = v_0 + (a (*) d)_m, a cyclic convolution of
// length R-1 of a_q = v[g^q] with d_j = e^{-2 pi i g^{-j} / R}, computed as a
// DFT, a pointwise product with dhat = DFT(d) / (R-1), and an inverse DFT
// (conjugate, DFT, conjugate).  X[0] is the plain sum v_0 + A_0.
//
// Rader stage for R = 73 (R - 1 = 72) with G lanes per butterfly, G in {2, 4, 8}.
// Lane s of a group holds the K = 72/G convolution inputs a[G j + s]; each
// length-72 DFT is a K-point DFT in registers, a twiddle e^{-2 pi i s k1/72},
// and a G-point DFT across the lanes (DPP moves).  The second DFT runs the
// same steps in the opposite order, so no data goes through LDS between the
// two.  tab holds dhat (72 values, DFT_72(d)/72) then e^{-2 pi i j/72}, j < 72.
// Every lane of a round runs the arithmetic (idle groups on zeros) so each
// lane move has its partner; rounds with no work at all are skipped.
// Rader permutation of the prime 73 for G lanes per butterfly, built by the
// compiler: lane s gathers inputs g^(s + G j) and scatters outputs to
// g^-(s + G kk), j, kk < 72 / G.
template <int G>
struct RaderIdx {
  int in[G][72 / G];
  int out[G][72 / G];
  constexpr RaderIdx() : in(), out() {
    const long g = ct_primroot(73), ginv = ct_powmod(g, 71, 73);
    for (int s = 0; s < G; ++s)
      for (int j = 0; j < 72 / G; ++j) {
        in[s][j] = int(ct_powmod(g, s + G * j, 73));
        out[s][j] = int(ct_powmod(ginv, s + G * j, 73));
      }
  }
};
template <int G>
struct RaderTab {
  static constexpr RaderIdx<G> t{};
};

// Entry J of row s of a Rader table for lane group index s < G (2 or 4): a
// blend of the row's compile-time entries by the bits of s.
template <int G, bool OUT, int J>
__device__ __forceinline__ int lane_entry(int s) {
  constexpr auto& t = OUT ? RaderTab<G>::t.out : RaderTab<G>::t.in;
  if constexpr (G == 2) {
    constexpr int a = t[0][J], d = t[1][J] - t[0][J];
    return a + s * d;
  } else {
    static_assert(G == 4, "two or four lanes");
    constexpr int a = t[0][J], d1 = t[1][J] - t[0][J], d2 = t[2][J] - t[0][J];
    constexpr int d3 = t[3][J] - t[2][J] - t[1][J] + t[0][J];
    const int b0 = s & 1, b1 = s >> 1;
    return a + b0 * d1 + b1 * d2 + (b0 & b1) * d3;
  }
}

// Gather of Rader inputs J.. of lane group s (compile-time recursion, so the
// permutation entries are constant expressions), with the stage twiddles
// when ns > 1.
template <typename T, int G, int K, int J, int ZP>
__device__ __forceinline__ void rader_gather(cx<T>* x, const cx<T>* Z, int b, int nbp, int p, int s, int ns, int k,
                                             const cx<T>* __restrict__ tw, bool act) {
  const int r = lane_entry<G, false, J>(s);
  cx<T> v = Z[(b + r * nbp) * ZP + p];
  if (ns > 1) v = cmul(v, tw[k * 72 + r - 1]);
  x[J].re = act ? v.re : T(0);
  x[J].im = act ? v.im : T(0);
  if constexpr (J + 1 < K) rader_gather<T, G, K, J + 1, ZP>(x, Z, b, nbp, p, s, ns, k, tw, act);
}

// Scatter of Rader outputs KK.. of lane group s to rows base + ns g^-(s + G kk).
template <typename T, int G, int K, int KK, int ZP>
__device__ __forceinline__ void rader_scatter(cx<T>* Z, const cx<T>* x, int base, int ns, int p, int s) {
  const int oi = lane_entry<G, true, KK>(s);
  Z[(base + oi * ns) * ZP + p] = x[KK];
  if constexpr (KK + 1 < K) rader_scatter<T, G, K, KK + 1, ZP>(Z, x, base, ns, p, s);
}

// ctab: the kernel spectrum and twiddles in LDS, laid out [k1][s] for this G
// (entry k1 G + s: dhat[k1 + K bitrev(s)], then 72 entries e^{-2 pi i s k1/72}),
// so each lane reads them at its own base plus immediate offsets; null: the
// global table tab (dhat[0..71], then e^{-2 pi i j/72}).
template <typename T, int NP, int NT, int PMAX, int G, int PC = 0, int NSC = 0, int ZP = NP>
__device__ __forceinline__ void stage_rader73(cx<T>* Z, int P_rt, int ns_rt, const cx<T>* __restrict__ tw,
                                              const cx<T>* __restrict__ tab, const cx<T>* ctab = nullptr) {
  static_assert(G == 2 || G == 4 || G == 8, "lanes per Rader butterfly");
  constexpr int R = 73, L = 72, K = L / G;
  constexpr int NBG = (((PC ? PC : PMAX) / R) * NP * G + NT - 1) / NT;
  const int P = PC ? PC : P_rt;
  const int ns = NSC ? NSC : ns_rt;
  constexpr long g = ct_primroot(R);
  constexpr int gG = int(ct_powmod(g, G, R));
  constexpr long ginv = ct_powmod(g, R - 2, R);
  constexpr int giG = int(ct_powmod(ginv, G, R));
  const cx<T>* dhat = tab;
  const cx<T>* w72 = tab + L;
  const int nbp = P / R;
  const int items = nbp * NP;
  const int tid = opaque_tid();
  const int s = tid & (G - 1);
  int gs = 1, gis = 1;  // g^s and g^{-s} mod R
  for (int e = 0; e < s; ++e) {
    gs = int((long(gs) * g) % R);
    gis = int((long(gis) * ginv) % R);
  }
  // one round: outputs stay in x; several rounds keep them in out
  cx<T> out[NBG > 1 ? NBG : 1][NBG > 1 ? K : 1];
  cx<T> out0[NBG];
  cx<T> x[K];
#pragma unroll
  for (int i = 0; i < NBG; ++i) {
    if (i * (NT / G) >= items) break;  // uniform over the block
    const int item = tid / G + i * (NT / G);
    const bool act = item < items;
    const int p = act ? item % NP : 0;
    const int b = act ? item / NP : 0;
    const int k = b % ns;
    // idle groups (b = p = 0) read valid entries and discard the results:
    // no request is predicated
    if constexpr (G <= 4) {
      rader_gather<T, G, K, 0, ZP>(x, Z, b, nbp, p, s, ns, k, tw, act);
    } else {
      int r = gs;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        cx<T> v = Z[(b + r * nbp) * ZP + p];
        if (ns > 1) v = cmul(v, tw[k * (R - 1) + r - 1]);
        x[j] = v;
        r = (r * gG) % R;
      }
    }
    cx<T> v0 = Z[b * ZP + p];
    v0.re = act ? v0.re : T(0);
    v0.im = act ? v0.im : T(0);
    // forward length-72 DFT of a
    dft_any<T, K>(x);
    // twiddles e^{-2 pi i s k1 / 72}: compile-time constants for two lanes
    // (identity on lane 0), a table otherwise
#pragma unroll
    for (int k1 = 1; k1 < K; ++k1) {
      if constexpr (G == 2) {
        const cx<T> w = {T(Tw<72>::t.c[k1]), T(-Tw<72>::t.s[k1])};
        const cx<T> y = cmul(x[k1], w);
        x[k1] = csel(s != 0, y, x[k1]);
      } else {
        x[k1] = cmul(x[k1], ctab ? ctab[72 + k1 * G + s] : w72[s * k1]);
      }
    }
    if constexpr (G >= 8) lane_radix2<T, K, 4, false>(x, s);
    if constexpr (G >= 4) lane_radix2<T, K, 2, false>(x, s);
    lane_radix2<T, K, 1, false>(x, s);
    // lane s holds A[k1 + K bitrev(s)]; X[0] = v0 + A[0] (lane 0, k1 = 0)
    const int k2 = lane_bitrev<G>(s);
    out0[i] = v0 + x[0];
#pragma unroll
    for (int k1 = 0; k1 < K; ++k1) x[k1] = conj(cmul(x[k1], ctab ? ctab[k1 * G + s] : dhat[k1 + K * k2]));
    // second length-72 DFT: across lanes first (bit-reversed in, natural out)
    lane_radix2<T, K, 1, true>(x, s);
    if constexpr (G >= 4) lane_radix2<T, K, 2, true>(x, s);
    if constexpr (G >= 8) lane_radix2<T, K, 4, true>(x, s);
#pragma unroll
    for (int j2 = 1; j2 < K; ++j2) {
      if constexpr (G == 2) {
        const cx<T> w = {T(Tw<72>::t.c[j2]), T(-Tw<72>::t.s[j2])};
        const cx<T> y = cmul(x[j2], w);
        x[j2] = csel(s != 0, y, x[j2]);
      } else {
        x[j2] = cmul(x[j2], ctab ? ctab[72 + j2 * G + s] : w72[j2 * s]);
      }
    }
    dft_any<T, K>(x);
    // lane s holds conj(c[s + G kk]);  X[g^{-(s + G kk)}] = v0 + c
#pragma unroll
    for (int kk = 0; kk < K; ++kk) x[kk] = v0 + conj(x[kk]);
    if constexpr (NBG > 1) {
#pragma unroll
      for (int kk = 0; kk < K; ++kk) out[i][kk] = x[kk];
    }
  }
  __syncthreads();
  const int tid2 = opaque_tid();
#pragma unroll
  for (int i = 0; i < NBG; ++i) {
    const int item = tid2 / G + i * (NT / G);
    if (item < items) {
      const int p = item % NP;
      const int b = item / NP;
      const int k = b % ns;
      const int base = (b - k) * R + k;
      if constexpr (G <= 4) {
        if constexpr (NBG > 1) rader_scatter<T, G, K, 0, ZP>(Z, out[i], base, ns, p, s);
        else rader_scatter<T, G, K, 0, ZP>(Z, x, base, ns, p, s);
      } else {
        int oi = gis;
#pragma unroll
        for (int kk = 0; kk < K; ++kk) {
          Z[(base + oi * ns) * ZP + p] = (NBG > 1) ? out[i][kk] : x[kk];
          oi = (oi * giG) % R;
        }
      }
      if (s == 0) Z[base * ZP + p] = out0[i];
    }
  }
  __syncthreads();
}

// Forward DFT of length P of every pair column of Z.
template <typename T, int NP, int NT, int PMAX, int RADER, int SLIM>
__device__ __forceinline__ void dft_engine(cx<T>* Z, int P, int nstages, const Stage* __restrict__ stp,
                                           const cx<T>* __restrict__ tw, const cx<T>* __restrict__ cs) {
  for (int s = 0; s < nstages; ++s) {
    const Stage st = stp[s];
    const cx<T>* t = tw + st.tw_off;
    switch (st.radix) {
      case 2: stage<T, 2, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul); break;
      case 3: stage<T, 3, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul); break;
      case 4: stage<T, 4, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul); break;
      case 5: stage<T, 5, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul); break;
      case 7: stage<T, 7, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul); break;
      case 8: stage<T, 8, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul); break;
      case 9: stage<T, 9, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul); break;
      case 11:
        if constexpr (SLIM != 1) stage<T, 11, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul);
        break;
      case 13:
        if constexpr (SLIM != 1) stage<T, 13, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul);
        break;
      // primes 17..31: only in the wide shapes (SLIM == 2)
      case 17:
        if constexpr (SLIM == 2) stage<T, 17, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul);
        break;
      case 19:
        if constexpr (SLIM == 2) stage<T, 19, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul);
        break;
      case 23:
        if constexpr (SLIM == 2) stage<T, 23, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul);
        break;
      case 29:
        if constexpr (SLIM == 2) stage<T, 29, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul);
        break;
      case 31:
        if constexpr (SLIM == 2) stage<T, 31, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul);
        break;
      case 14:
        // only after a Rader stage (1022 = 73 x 14): one LDS sweep instead of 7 and 2
        if constexpr (RADER != 0) stage<T, 14, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul);
        break;
      case 16: stage<T, 16, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul); break;
      case 32:
        // largest power-of-two codelet: 32 in FP32 only (keeps FP64 threads
        // near 100 registers, so two workgroups share a CU)
        if constexpr (sizeof(T) == 4) stage<T, 32, NP, NT, PMAX>(Z, P, st.ns, t, st.ns_mul);
        break;
      case 73:
        if constexpr (RADER != 0) stage_rader73<T, NP, NT, PMAX, RADER>(Z, P, st.ns, t, cs + st.cs_off);
        break;
      default: break;  // the planner only emits the radices above
    }
  }
}

// Stage list of a kernel specialised for one DFT work length: radices in
// Stockham order.  StageList<> means the run-time list of the description.
template <int... Rs>
struct StageList {
  static constexpr int count = sizeof...(Rs);
};

// Compile-time Stockham engine: stage stride NS and twiddle offset TWOFF
// accumulate as the host builds them (ns * (R - 1) twiddles per stage, the
// Rader constants first in the constant table).
template <typename T, int NP, int ZP, int NT, int RADER, int P, int NS, int TWOFF, int R, int... Rest>
__device__ __forceinline__ void dft_engine_ct(cx<T>* Z, const cx<T>* __restrict__ tw, const cx<T>* __restrict__ cs,
                                              const cx<T>* __restrict__ ctab) {
  if constexpr (R == 73) {
    static_assert(RADER != 0, "Rader stage needs a Rader kernel shape");
    stage_rader73<T, NP, NT, P, RADER, P, NS, ZP>(Z, P, NS, tw + TWOFF, cs, ctab);
  } else {
    stage<T, R, NP, NT, P, P, NS, ZP>(Z, P, NS, tw + TWOFF);
  }
  if constexpr (sizeof...(Rest) > 0)
    dft_engine_ct<T, NP, ZP, NT, RADER, P, NS * R, TWOFF + NS * (R - 1), Rest...>(Z, tw, cs, ctab);
}

template <typename T, int NP, int ZP, int NT, int RADER, int P, int... Rs>
__device__ __forceinline__ void dft_engine_list(cx<T>* Z, const cx<T>* __restrict__ tw, const cx<T>* __restrict__ cs,
                                                const cx<T>* __restrict__ ctab, StageList<Rs...>) {
  dft_engine_ct<T, NP, ZP, NT, RADER, P, 1, 0, Rs...>(Z, tw, cs, ctab);
}

// Element k of the length-M DFT of pair p after dft_full.
template <typename T, int ZP, class AX>
__device__ __forceinline__ cx<T> dft_result(const cx<T>* Z, const AX& ax, int k, int p) {
  cx<T> z = Z[k * ZP + p];
  if (ax.blue()) z = cmul(conj(z), static_cast<const cx<T>*>(ax.d.chirp)[k]);
  return z;
}

// ----------------------------------------------------------------------------- tile access

// Real tile X: element j of line t of the tile at X[j * XP + t] (lines
// innermost, for any axis; XP = 2 ZP >= TL), which is also the packed
// complex layout Z[m * ZP + p] with line t = 2p + w in component w.
template <int XP>
__device__ __forceinline__ int xi(int t, int j) {
  return j * XP + t;
}

// Halfcomplex entry k (complex X_k) of a real DFT stored as h[0..n-1].
template <typename T, int XP>
__device__ __forceinline__ cx<T> hc_get(const T* X, int t, int k, int n) {
  if (k == 0) return {X[xi<XP>(t, 0)], T(0)};
  if (2 * k < n) return {X[xi<XP>(t, k)], X[xi<XP>(t, n - k)]};
  if (2 * k == n) return {X[xi<XP>(t, k)], T(0)};
  return {X[xi<XP>(t, n - k)], -X[xi<XP>(t, k)]};
}

// DCT-II reorder: v_m = x_{perm(m)} (even indices ascending, then odd descending).
__device__ __forceinline__ int perm_even_odd(int m, int n) {
  return (2 * m <= n - 1) ? 2 * m : 2 * (n - 1 - m) + 1;
}

// Packing: the complex input of the length-M DFT for pair p at index m
// (times the chirp for Bluestein, conjugated for inverse kinds).
template <typename T, int XP, int kind, class AX>
__device__ __forceinline__ cx<T> pack_value(const T* X, const AX& ax, int m, int p) {
  const int n = ax.n(), M = ax.M();
  const int t0 = 2 * p, t1 = 2 * p + 1;
  cx<T> val = {T(0), T(0)};
  if (m >= M) return val;
  switch (kind) {
    case K_R2HC:
      val = {X[xi<XP>(t0, m)], X[xi<XP>(t1, m)]};
      break;
    case K_DCT2:
    case K_DST2: {
      const int j = perm_even_odd(m, n);
      val = {X[xi<XP>(t0, j)], X[xi<XP>(t1, j)]};
      if (kind == K_DST2 && (j & 1)) val = {-val.re, -val.im};
      break;
    }
    case K_DCT1: {
      const int j = (m < n) ? m : M - m;
      val = {X[xi<XP>(t0, j)], X[xi<XP>(t1, j)]};
      break;
    }
    case K_DST1: {
      if (m == 0 || m == n + 1) break;
      if (m <= n) {
        val = {X[xi<XP>(t0, m - 1)], X[xi<XP>(t1, m - 1)]};
      } else {
        const int j = M - m - 1;
        val = {-X[xi<XP>(t0, j)], -X[xi<XP>(t1, j)]};
      }
      break;
    }
    case K_HC2R: {
      const cx<T> a = hc_get<T, XP>(X, t0, m, n);
      const cx<T> b = hc_get<T, XP>(X, t1, m, n);
      val = {a.re - b.im, -(a.im + b.re)};  // conj(a + i b)
      break;
    }
    case K_DST4:
    case K_DCT4: {
      // z_m e^{-i pi m/(2n)} for m < n, zero-padded to the DFT length 2n
      if (m < n) {
        const cx<T> z = {X[xi<XP>(t0, m)], X[xi<XP>(t1, m)]};
        val = cmul(z, static_cast<const cx<T>*>(ax.d.pre)[m]);
      }
      break;
    }
    case K_DCT3:
    case K_DST3: {
      // V_k = e^{+i pi k/(2n)} (c_k - i c_{n-k}), c_n = 0; DST3 reverses c first.
      const int k = m;
      const int ka = (kind == K_DST3) ? n - 1 - k : k;
      const T c0k = X[xi<XP>(t0, ka)], c1k = X[xi<XP>(t1, ka)];
      T c0n = T(0), c1n = T(0);
      if (k > 0) {
        const int kb = (kind == K_DST3) ? k - 1 : n - k;
        c0n = X[xi<XP>(t0, kb)];
        c1n = X[xi<XP>(t1, kb)];
      }
      const cx<T> e = conj(static_cast<const cx<T>*>(ax.d.pre)[k]);
      const cx<T> v0 = cmul(e, cx<T>{c0k, -c0n});
      const cx<T> v1 = cmul(e, cx<T>{c1k, -c1n});
      val = {v0.re - v1.im, -(v0.im + v1.re)};  // conj(v0 + i v1)
      break;
    }
    default:
      break;
  }
  if (ax.blue()) val = cmul(val, static_cast<const cx<T>*>(ax.d.chirp)[m]);
  return val;
}

// Unpacking: output coefficient k of line t from the DFT result.
template <typename T, int ZP, int kind, class AX>
__device__ __forceinline__ T unpack_value(const cx<T>* Z, const AX& ax, int t, int k) {
  const int n = ax.n(), M = ax.M();
  const int p = t >> 1, w = t & 1;
  switch (kind) {
    case K_R2HC:
    case K_DCT2:
    case K_DST2: {
      int kk = k;
      if (kind == K_R2HC && 2 * k > n) kk = n - k;
      if (kind == K_DST2) kk = n - 1 - k;
      const cx<T> zk = dft_result<T, ZP>(Z, ax, kk, p);
      const cx<T> zr = conj(dft_result<T, ZP>(Z, ax, kk == 0 ? 0 : M - kk, p));
      // line 0: (zk + zr)/2 ; line 1: (zk - zr)/(2i)
      cx<T> V;
      if (w == 0) V = {T(0.5) * (zk.re + zr.re), T(0.5) * (zk.im + zr.im)};
      else V = {T(0.5) * (zk.im - zr.im), -T(0.5) * (zk.re - zr.re)};
      if (kind == K_R2HC) return (2 * k <= n) ? V.re : V.im;
      const cx<T> e = static_cast<const cx<T>*>(ax.d.pre)[kk];
      return T(2) * (e.re * V.re - e.im * V.im);
    }
    case K_DCT1: {
      const cx<T> z = dft_result<T, ZP>(Z, ax, k, p);
      return w ? z.im : z.re;
    }
    case K_DST1: {
      const cx<T> z = dft_result<T, ZP>(Z, ax, k + 1, p);
      return w ? z.re : -z.im;
    }
    case K_HC2R: {
      const cx<T> z = dft_result<T, ZP>(Z, ax, k, p);
      return w ? -z.im : z.re;
    }
    case K_DST4:
    case K_DCT4: {
      // Q_k = e^{-i pi (2k+1)/(4n)} Z_k; with k' = 2n-1-k, Q_k - Q_k' carries the
      // DCT-IV of both lines (real: line 0, imaginary: line 1) and Q_k + Q_k'
      // the DST-IV (line 0: minus the imaginary part, line 1: the real part)
      const cx<T>* pre = static_cast<const cx<T>*>(ax.d.pre);
      const cx<T> pk = cmul(pre[k], pre[n]);  // e^{-i pi (2k+1)/(4n)}; pre[n] = e^{-i pi/(4n)}
      const cx<T> pk2 = {-pk.re, pk.im};      // e^{-i pi (2k'+1)/(4n)} = -conj(pk)
      const cx<T> Qk = cmul(pk, dft_result<T, ZP>(Z, ax, k, p));
      const cx<T> Qk2 = cmul(pk2, dft_result<T, ZP>(Z, ax, M - 1 - k, p));
      if (kind == K_DCT4) return w ? (Qk.im - Qk2.im) : (Qk.re - Qk2.re);
      return w ? (Qk.re + Qk2.re) : -(Qk.im + Qk2.im);
    }
    case K_DCT3:
    case K_DST3: {
      const int q = (k & 1) ? n - 1 - (k >> 1) : (k >> 1);
      const cx<T> z = dft_result<T, ZP>(Z, ax, q, p);
      T v = w ? -z.im : z.re;
      if (kind == K_DST3 && (k & 1)) v = -v;
      return v;
    }
    default:
      return T(0);
  }
}

// X (real tile) -> Z (packed complex), through registers.
template <typename T, int NP, int NT, int PMAX, int kind, class AX, int ZP = NP>
__device__ __forceinline__ void pack_k(T* X, cx<T>* Z, const AX& ax) {
  constexpr int XP = 2 * ZP;
  constexpr int E = ((AX::ct ? AX::Pc : PMAX) * NP + NT - 1) / NT;
  const int items = ax.P() * NP;
  const int tid = opaque_tid();
  cx<T> v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int item = tid + i * NT;
    if (item < items) v[i] = pack_value<T, XP, kind>(X, ax, item / NP, item % NP);
  }
  __syncthreads();
  const int tid2 = opaque_tid();
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int item = tid2 + i * NT;
    if (item < items) Z[(item / NP) * ZP + item % NP] = v[i];
  }
  __syncthreads();
}

template <typename T, int NP, int NT, int PMAX, class AX>
__device__ __forceinline__ void pack(T* X, cx<T>* Z, int kind, const AX& ax) {
  switch (kind) {
    case K_R2HC: pack_k<T, NP, NT, PMAX, K_R2HC>(X, Z, ax); break;
    case K_HC2R: pack_k<T, NP, NT, PMAX, K_HC2R>(X, Z, ax); break;
    case K_DCT2: pack_k<T, NP, NT, PMAX, K_DCT2>(X, Z, ax); break;
    case K_DCT3: pack_k<T, NP, NT, PMAX, K_DCT3>(X, Z, ax); break;
    case K_DST2: pack_k<T, NP, NT, PMAX, K_DST2>(X, Z, ax); break;
    case K_DST3: pack_k<T, NP, NT, PMAX, K_DST3>(X, Z, ax); break;
    case K_DCT1: pack_k<T, NP, NT, PMAX, K_DCT1>(X, Z, ax); break;
    case K_DST4:
    case K_DCT4: pack_k<T, NP, NT, PMAX, K_DCT4>(X, Z, ax); break;  // same pre-step
    default: pack_k<T, NP, NT, PMAX, K_DST1>(X, Z, ax); break;
  }
}

// Z -> X, through registers, optionally dividing by the eigenvalue sum.
template <typename T, int NP, int NT, int PMAX, int kind, class AX, int ZP = NP>
__device__ __forceinline__ void unpack_k(cx<T>* Z, T* X, const AX& ax, const PassArgs& a,
                                         int64_t l0, bool scale, const T* lts = nullptr) {
  constexpr int TL = 2 * NP;
  constexpr int XP = 2 * ZP;
  constexpr int E = ((AX::ct ? AX::Nc : PMAX) * TL + NT - 1) / NT;
  static_assert(NT % TL == 0, "thread count must be a multiple of the tile width");
  const int n = ax.n();
  const int items = n * TL;
  const int tid = opaque_tid();
  const int t = tid % TL;  // fixed per thread
  T lam_other = T(0);
  bool zero_line = false;  // the all-zero mode of a singular problem lives on line 0
  bool dead_line = false;  // padding line of a partial tile: holds zeros, must stay finite
  if (scale) {
    const int64_t l = l0 + t;
    const T* la = static_cast<const T*>(a.lam_a);
    const T* lb = static_cast<const T*>(a.lam_b);
    if (l < a.nlines) {
      if (lb) lam_other = la[l / a.nb] + lb[l % a.nb];
      else if (la) lam_other = la[l];
    } else {
      dead_line = true;
    }
    zero_line = a.singular && (l == 0);
  }
  const T* lt = static_cast<const T*>(a.lam_this);
  T v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int item = tid + i * NT;
    if (item < items) {
      const int k = item / TL;
      T x = unpack_value<T, ZP, kind>(Z, ax, t, k);
      if (scale) {
        const bool zero = dead_line || (zero_line && k == 0);
        if constexpr (AX::ct) x = zero ? T(0) : quick_div(x, lam_other + (lts ? lts[k] : lt[k]));
        else x = zero ? T(0) : x / (lam_other + lt[k]);
      }
      v[i] = x;
    }
  }
  __syncthreads();
  const int tid2 = opaque_tid();
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int item = tid2 + i * NT;
    if (item < items) X[xi<XP>(tid2 % TL, item / TL)] = v[i];
  }
  __syncthreads();
}

template <typename T, int NP, int NT, int PMAX, class AX>
__device__ __forceinline__ void unpack(cx<T>* Z, T* X, int kind, const AX& ax,
                                       const PassArgs& a, int64_t l0, bool scale) {
  switch (kind) {
    case K_R2HC: unpack_k<T, NP, NT, PMAX, K_R2HC>(Z, X, ax, a, l0, scale); break;
    case K_HC2R: unpack_k<T, NP, NT, PMAX, K_HC2R>(Z, X, ax, a, l0, scale); break;
    case K_DCT2: unpack_k<T, NP, NT, PMAX, K_DCT2>(Z, X, ax, a, l0, scale); break;
    case K_DCT3: unpack_k<T, NP, NT, PMAX, K_DCT3>(Z, X, ax, a, l0, scale); break;
    case K_DST2: unpack_k<T, NP, NT, PMAX, K_DST2>(Z, X, ax, a, l0, scale); break;
    case K_DST3: unpack_k<T, NP, NT, PMAX, K_DST3>(Z, X, ax, a, l0, scale); break;
    case K_DCT1: unpack_k<T, NP, NT, PMAX, K_DCT1>(Z, X, ax, a, l0, scale); break;
    case K_DST4: unpack_k<T, NP, NT, PMAX, K_DST4>(Z, X, ax, a, l0, scale); break;
    case K_DCT4: unpack_k<T, NP, NT, PMAX, K_DCT4>(Z, X, ax, a, l0, scale); break;
    default: unpack_k<T, NP, NT, PMAX, K_DST1>(Z, X, ax, a, l0, scale); break;
  }
}

// ----------------------------------------------------------------------------- strided-tile shortcuts
// For a strided tile the real tile X[j * TL + t] and the packed work buffer
// Z[m * NP + p] (line t = 2p + w in component w) are the same memory.  A
// DCT-I input then only needs its even extension, rows m = n..M-1 copied from
// rows M - m, and a DCT-I output is already in place.
template <typename T, int NP, int NT, int ZP = NP>
__device__ __forceinline__ void dct1_mirror(cx<T>* Z, int n, int M) {
  const int items = (M - n) * NP;
  for (int it = int(threadIdx.x); it < items; it += NT) {
    const int m = n + it / NP, p = it % NP;
    Z[m * ZP + p] = Z[(M - m) * ZP + p];
  }
  __syncthreads();
}

// In-place division of a DCT-I result by the eigenvalue sums, written to the
// mirrored rows as well, so that the result is at once the input of the
// inverse DCT-I.
// lts: the eigenvalues of this axis staged in LDS by a specialised kernel
// (else null: read from global memory).  Specialised kernels (compile-time
// length) divide with quick_div, the generic shapes with IEEE division.
template <typename T, int NP, int NT, class AX, int ZP = NP>
__device__ __forceinline__ void dct1_scale_mirror(T* X, const AX& ax, const PassArgs& a, int64_t l0,
                                                  const T* lts = nullptr) {
  constexpr int TL = 2 * NP;
  constexpr int XP = 2 * ZP;
  static_assert(NT % TL == 0, "thread count must be a multiple of the tile width");
  const int n = ax.n(), M = ax.M();
  const int tid = int(threadIdx.x);
  const int t = tid % TL;
  const int64_t l = l0 + t;
  const T* la = static_cast<const T*>(a.lam_a);
  const T* lb = static_cast<const T*>(a.lam_b);
  const T* lt = static_cast<const T*>(a.lam_this);
  T lam_other = T(0);
  const bool dead_line = l >= a.nlines;
  if (!dead_line) {
    if (lb) lam_other = la[l / a.nb] + lb[l % a.nb];
    else if (la) lam_other = la[l];
  }
  const bool zero_line = a.singular && (l == 0);
  if constexpr (AX::ct) {
    const T* lk = lts ? lts : lt;
#pragma unroll 4
    for (int it = tid; it < n * TL; it += NT) {
      const int k = it / TL;
      const int xi_k = k * XP + t;
      const T x = (dead_line || (zero_line && k == 0)) ? T(0) : quick_div(X[xi_k], lam_other + lk[k]);
      X[xi_k] = x;
      if (k >= 1 && k <= n - 2) X[(M - k) * XP + t] = x;
    }
  } else {
    for (int it = tid; it < n * TL; it += NT) {
      const int k = it / TL;
      const int xi_k = k * XP + t;
      const T x = (dead_line || (zero_line && k == 0)) ? T(0) : X[xi_k] / (lam_other + lt[k]);
      X[xi_k] = x;
      if (k >= 1 && k <= n - 2) X[(M - k) * XP + t] = x;
    }
  }
  __syncthreads();
}

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD
// b mod 8).  Give each XCD a contiguous range of tiles, so that neighbouring
// tiles -- which share cache lines on the strided axes -- meet in the same L2.
// A bijection of [0, G) for any G.
__device__ __forceinline__ int64_t xcd_tile(unsigned b, unsigned G) {
  constexpr unsigned kXcd = 8;
  const unsigned q = G / kXcd, r = G % kXcd;
  const unsigned x = b % kXcd, i = b / kXcd;
  return int64_t(x) * q + (x < r ? x : r) + i;
}

// One transform phase of a sweep (forward, or the inverse after the
// eigenvalue division): pack, DFT (or Bluestein convolution), unpack.  K is
// the compile-time kind of a specialised kernel, or -2 for the run-time kind.
template <typename T, int NP, int NT, int PMAX, int RADER, int SLIM, class AX, class ST, int K, int ZP>
__device__ __forceinline__ void transform_phase(T* X, cx<T>* Z, const AX& ax, const PassArgs& a, int64_t l0,
                                                int kind_rt, bool scale, int kind_next, bool& mirrored,
                                                const T* lts = nullptr, const cx<T>* ctab = nullptr) {
  const int kind = K >= 0 ? K : kind_rt;
  const cx<T>* tw = static_cast<const cx<T>*>(ax.d.tw);
  const cx<T>* cs = static_cast<const cx<T>*>(ax.d.cs);
  // without a chirp convolution the in-place shortcuts apply
  const bool inplace = !ax.blue();
  if (inplace && kind == K_DCT1) {
    if (!mirrored) dct1_mirror<T, NP, NT, ZP>(Z, ax.n(), ax.M());
  } else if (!(inplace && kind == K_R2HC)) {
    if constexpr (K >= 0) pack_k<T, NP, NT, PMAX, K, AX, ZP>(X, Z, ax);
    else pack<T, NP, NT, PMAX>(X, Z, kind, ax);
  }
  // Stockham DFT; for Bluestein: DFT, times the kernel spectrum, conjugate, DFT
  // (the unpacker conjugates and applies the chirp).  The two DFTs share one
  // copy of the engine code (run-time loop).
  const int nrep = ax.blue() ? 2 : 1;
  for (int rep = 0; rep < nrep; ++rep) {
    if (rep == 1) {
      const cx<T>* bh = static_cast<const cx<T>*>(ax.d.bhat);
      const int items = ax.P() * NP;
      for (int item = threadIdx.x; item < items; item += NT) {
        const int zi = (item / NP) * ZP + item % NP;
        Z[zi] = conj(cmul(Z[zi], bh[item / NP]));
      }
      __syncthreads();
    }
    if constexpr (ST::count > 0) dft_engine_list<T, NP, ZP, NT, RADER, AX::Pc>(Z, tw, cs, ctab, ST{});
    else dft_engine<T, NP, NT, PMAX, RADER, SLIM>(Z, ax.P(), ax.d.nstages, ax.d.st, tw, cs);
  }
  if (inplace && kind == K_DCT1) {
    if (scale) {
      dct1_scale_mirror<T, NP, NT, AX, ZP>(X, ax, a, l0, lts);
      mirrored = kind_next == K_DCT1;
    }
  } else {
    if constexpr (K >= 0) unpack_k<T, NP, NT, PMAX, K, AX, ZP>(Z, X, ax, a, l0, scale, lts);
    else unpack<T, NP, NT, PMAX>(Z, X, kind, ax, a, l0, scale);
  }
}


// Bytes of LDS a specialised kernel uses for its tile / work buffer (the
// larger of n real rows and P complex rows at pitch ZP), rounded to 16.
template <typename T, int N, int P, int ZP>
constexpr int spec_main_lds() {
  const int xs = 2 * ZP * N, zs = 2 * ZP * P;
  return ((xs > zs ? xs : zs) * int(sizeof(T)) + 15) / 16 * 16;
}

// LDS of a specialised kernel behind the tile: the Rader constants (144
// complex values) of a kernel with a Rader stage.
template <typename T, int RADER>
constexpr int spec_ctab_lds() {
  return RADER ? 144 * 2 * int(sizeof(T)) : 0;
}

// Whether a fused specialised kernel stages the axis's eigenvalues in LDS:
// only when that does not cost a second workgroup per CU (160 KB of LDS).
template <typename T, int N, int P, int ZP, int RADER>
constexpr bool spec_stage_lam() {
  constexpr int half = 80 * 1024;
  constexpr int base = spec_main_lds<T, N, P, ZP>() + spec_ctab_lds<T, RADER>();
  return base + N * int(sizeof(T)) <= half || base > half;
}

// ----------------------------------------------------------------------------- projection step I/O
// Quotient and remainder of a non-negative 64-bit index, in 32-bit arithmetic
// when both operands allow it.
__device__ __forceinline__ void idx_divmod(int64_t x, int64_t d, int64_t* q, int64_t* r) {
  if (((x | d) >> 31) == 0) {
    const uint32_t qq = uint32_t(x) / uint32_t(d);
    *q = qq;
    *r = uint32_t(x) - qq * uint32_t(d);
  } else {
    *q = x / d;
    *r = x - *q * d;
  }
}

// First pass of a projection step (along the last padded axis): element j of
// line l is div(vel) / adt at cell (l / n1, l % n1, j), summed in FP64 over
// the velocity components present.  Lanes take consecutive j of one line, so
// the three component reads are coalesced; each thread issues the face reads
// of PDU elements before it uses any of them (more requests in flight).
// Cell coordinates (c0, c1) of line l0 + t, from those of the tile's first
// line (lines run over axis 1 fastest; a division only where t wraps it).
__device__ __forceinline__ void line_cell(int64_t c0_0, int64_t c1_0, int t, int64_t n1, int64_t* c0, int64_t* c1) {
  int64_t a1 = c1_0 + t, a0 = c0_0;
  if (a1 >= n1) {
    const int64_t k = a1 / n1;
    a0 += k;
    a1 -= k * n1;
  }
  *c0 = a0;
  *c1 = a1;
}

template <typename T, typename S, int TL, int NT, int XP>
__device__ __forceinline__ void proj_div_load(T* X, const PassArgs& a, int64_t l0, int n) {
  constexpr int PDU = 4;
  const ProjDev& q = a.proj;
  const int total = TL * n;
  int64_t c0_0, c1_0;
  idx_divmod(l0, q.n[1], &c0_0, &c1_0);
  for (int e0 = int(threadIdx.x); e0 < total; e0 += PDU * NT) {
    // faces below and above each of the PDU cells, per component (zeros for
    // absent components and for elements past the tile or the last line)
    S lo[PDU][3], hi[PDU][3];
#pragma unroll
    for (int i = 0; i < PDU; ++i) {
      const int e = e0 + i * NT;
      const int t = e / n, j = e - t * n;
      const bool ok = e < total && l0 + t < a.nlines;
      int64_t c[3];
      line_cell(c0_0, c1_0, ok ? t : 0, q.n[1], &c[0], &c[1]);
      c[2] = ok ? j : 0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const S* u = static_cast<const S*>(q.vel[d]);
        lo[i][d] = S(0);
        hi[i][d] = S(0);
        if (!u || !ok) continue;
        const int64_t o = c[0] * q.vs[d][0] + c[1] * q.vs[d][1] + c[2] * q.vs[d][2];
        // the face above cell c; on a periodic axis face n is face 0
        const int64_t up = (q.ext[d] == 0 && c[d] + 1 == q.n[d]) ? o - (q.n[d] - 1) * q.vs[d][d] : o + q.vs[d][d];
        lo[i][d] = u[o];
        hi[i][d] = u[up];
      }
    }
#pragma unroll
    for (int i = 0; i < PDU; ++i) {
      const int e = e0 + i * NT;
      if (e >= total) break;
      const int t = e / n, j = e - t * n;
      double sum = 0.0;
      if (l0 + t < a.nlines) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
          if (q.vel[d]) sum += (double(hi[i][d]) - double(lo[i][d])) * q.inv_h[d];
        sum *= q.inv_adt;
      }
      X[j * XP + t] = T(sum);
    }
  }
}

// Last pass of a projection step: phi (C order) is stored, added to the
// pressure, and the velocity component along the pass axis is corrected on
// its faces from the phi values of the same line (u -= adt grad phi; a
// Neumann boundary face keeps its value).
template <typename T, typename D, int TL, int NT, int XP>
__device__ __forceinline__ void proj_store(const T* X, const PassArgs& a, int64_t l0, int n) {
  const ProjDev& q = a.proj;
  D* phi = static_cast<D*>(a.dst);
  D* p = static_cast<D*>(q.p);
  D* w = static_cast<D*>(q.vel[2]);
  const int nf = n + q.ext[2];
  const double cw = q.adt * q.inv_h[2];
  const int total = TL * nf;
  int64_t c0_0, c1_0;
  idx_divmod(l0, q.n[1], &c0_0, &c1_0);
  // PSU elements per thread at a time: the reads of p and of the faces of w
  // for all of them are issued before any of them is updated
  constexpr int PSU = 4;
  for (int e0 = int(threadIdx.x); e0 < total; e0 += PSU * NT) {
    D pv[PSU], wv[PSU];
    int64_t ow[PSU];
#pragma unroll
    for (int i = 0; i < PSU; ++i) {
      const int e = e0 + i * NT;
      const int t = e / nf, f = e - t * nf;
      const bool ok = e < total && l0 + t < a.nlines;
      pv[i] = D(0);
      wv[i] = D(0);
      ow[i] = -1;
      if (!ok) continue;
      if (f < n) pv[i] = p[(l0 + t) * int64_t(n) + f];
      // a Dirichlet boundary face is corrected, a Neumann one keeps its value
      const bool upd = q.ext[2] == 0 || (f == 0 ? q.dlo[2] != 0 : f == n ? q.dhi[2] != 0 : true);
      if (w && upd) {
        int64_t c0, c1;
        line_cell(c0_0, c1_0, t, q.n[1], &c0, &c1);
        ow[i] = c0 * q.vs[2][0] + c1 * q.vs[2][1] + f;
        wv[i] = w[ow[i]];
      }
    }
#pragma unroll
    for (int i = 0; i < PSU; ++i) {
      const int e = e0 + i * NT;
      if (e >= total) break;
      const int t = e / nf, f = e - t * nf;
      if (l0 + t >= a.nlines) continue;
      if (f < n) {
        const double x = double(X[f * XP + t]);
        const int64_t o = (l0 + t) * int64_t(n) + f;
        phi[o] = D(x);
        p[o] = D(double(pv[i]) + x);
      }
      if (ow[i] >= 0) {
        double g;
        if (q.ext[2] == 0) g = double(X[f * XP + t]) - double(X[(f == 0 ? n - 1 : f - 1) * XP + t]);
        else if (f == 0) g = 2.0 * double(X[t]);
        else if (f == n) g = -2.0 * double(X[(n - 1) * XP + t]);
        else g = double(X[f * XP + t]) - double(X[(f - 1) * XP + t]);
        w[ow[i]] = D(double(wv[i]) - cw * g);
      }
    }
  }
}

// One sweep over tile `tile`.  AX, KF, KB, ST: length view, forward and
// inverse kinds (-1: no inverse) and stage list of a kernel specialised for
// one transform (Ax<>, -2, -2, StageList<>: everything from the description).
// ZP: LDS row pitch in complex values (NP for the generic shapes).
// PROJ: the kernel also serves the first and last passes of a projection step
// (a separate instantiation, so that the other kernels carry none of its code).
template <typename T, int NP, int NT, int PMAX, int RADER, int SLIM, class AX = Ax<>, int KF = -2, int KB = -2,
          class ST = StageList<>, int ZP = NP, bool PROJ = false>
__device__ __forceinline__ void line_pass_body(const PassArgs& a, int64_t tile, unsigned char* smem) {
  static_assert(ZP == NP || (KF >= 0 && ST::count > 0 && AX::ct), "a padded pitch needs a specialised kernel");
  constexpr int TL = 2 * NP;
  constexpr int XP = 2 * ZP;
  T* X = reinterpret_cast<T*>(smem);
  cx<T>* Z = reinterpret_cast<cx<T>*>(smem);
  const AX ax{a.ax};
  const int n = ax.n();
  const int64_t B = a.inner;
  const int64_t l0 = tile * TL;

  // Tile I/O of a specialised kernel (compile-time n) whose tile lies in one
  // plane of the array (B % TL == 0, or B == 1: the contiguous axis) and whose
  // byte offsets fit 32 bits: every element of the thread is requested before
  // the first LDS write, from a uniform tile base pointer and 32-bit lane
  // offsets.  Contiguous axis: the TL lines are TL * n consecutive elements,
  // read by consecutive lanes (fully coalesced) and transposed into LDS
  // through the padded pitch.  Strided axes: lanes take TL adjacent lines of
  // one row (TL consecutive elements), rows NT / TL apart per request.
  constexpr bool kFast = AX::ct && (TL * AX::Nc) % NT == 0;
  constexpr int EF = kFast ? TL * AX::Nc / NT : 1;  // elements per thread
  int mode = 0;       // 0 generic, 1 contiguous fast path, 2 strided fast path
  int64_t tbase = 0;  // element offset of the tile's first element
  if constexpr (kFast) {
    const bool full = l0 + TL <= a.nlines && a.contig;
    constexpr int64_t kLim = int64_t(1) << 29;  // elements: byte offsets of 8-byte values stay below 2^32
    if (B == 1) {
      mode = (full && int64_t(TL) * n < kLim) ? 1 : 0;
      tbase = l0 * n;
    } else {
      mode = (full && B % TL == 0 && int64_t(n) * B < kLim) ? 2 : 0;
      tbase = (l0 / B) * (int64_t(n) * B) + (l0 % B);
    }
  }
  const uint32_t Bu = uint32_t(B);
  // element e of this thread: 32-bit element offset from the tile base and LDS index
  auto off_c = [&](int tid, int e) { return uint32_t(tid + e * NT); };
  auto xi_c = [&](int tid, int e) {
    const int q = tid + e * NT;
    return (q % (AX::ct ? AX::Nc : 1)) * XP + q / (AX::ct ? AX::Nc : 1);
  };
  auto off_s = [&](int tid, int e) { return uint32_t(tid / TL + e * (NT / TL)) * Bu + uint32_t(tid % TL); };
  auto xi_s = [&](int tid, int e) { return (tid / TL + e * (NT / TL)) * XP + tid % TL; };

  // ---- load.  Generic path: thread (t, j0) reads elements j0, j0 + NT/TL,
  // ... of line t (lines innermost in LDS, conflict-free writes), CH at a
  // time, all CH before any LDS write; elements outside the array are read
  // from its first element and replaced by zeros, so no request is
  // predicated.  The element type of the source is a uniform branch around
  // whole loops.
  constexpr int ELD = (2 * NP * (AX::ct ? AX::Nc : PMAX) + NT - 1) / NT;  // bound for n <= PMAX
  constexpr int CH = ELD < 16 ? ELD : 16;
  auto fast_load = [&](auto src_elem, auto off, auto xi) {
    using S = decltype(src_elem);
    const int tid = opaque_tid();
    const char* sb = reinterpret_cast<const char*>(static_cast<const S*>(a.src) + tbase);
    S ld[EF];
#pragma unroll
    for (int e = 0; e < EF; ++e) ld[e] = *reinterpret_cast<const S*>(sb + off(tid, e) * uint32_t(sizeof(S)));
#pragma unroll
    for (int e = 0; e < EF; ++e) X[xi(tid, e)] = T(ld[e]);
  };
  auto generic_load = [&](auto src_elem) {
    using S = decltype(src_elem);
    const S* src = static_cast<const S*>(a.src);
    const int tid = opaque_tid();
    const int t = tid % TL;
    const int64_t l = l0 + t;
    const bool ok = l < a.nlines;
    const int64_t base = ok ? (l / a.src_vnb) * a.src_va + (l % a.src_vnb) * a.src_vb : 0;
    const int64_t sd = a.src_vd;
    for (int c = 0; c < ELD && c * (NT / TL) < n; c += CH) {
      S ld[CH];
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int j = tid / TL + (c + i) * (NT / TL);
        ld[i] = src[(ok && j < n) ? base + int64_t(j) * sd : base];
      }
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int j = tid / TL + (c + i) * (NT / TL);
        if (j < n) X[j * XP + t] = ok ? T(ld[i]) : T(0);
      }
    }
  };
  // a fused specialised kernel keeps this axis's eigenvalues in LDS behind
  // the tile (spec_main_lds bytes in)
  // and a kernel with a Rader stage its constants, in lane order (after the
  // 144 entries of the global layout: the G = 2 block, then the G = 4 block)
  T* lts = nullptr;
  cx<T>* ctab = nullptr;
  if constexpr (AX::ct && RADER != 0) {
    static_assert(RADER == 2 || RADER == 4, "lane-ordered Rader constants exist for 2 and 4 lanes");
    ctab = reinterpret_cast<cx<T>*>(smem + spec_main_lds<T, AX::Nc, AX::Pc, ZP>());
    const cx<T>* src = static_cast<const cx<T>*>(a.ax.cs) + (RADER == 2 ? 144 : 288);
    for (int i = int(threadIdx.x); i < 144; i += NT) ctab[i] = src[i];
  }
  if constexpr (AX::ct && KB >= 0 && spec_stage_lam<T, AX::Nc, AX::Pc, ZP, RADER>()) {
    lts = reinterpret_cast<T*>(smem + spec_main_lds<T, AX::Nc, AX::Pc, ZP>() + spec_ctab_lds<T, RADER>());
    const T* lt = static_cast<const T*>(a.lam_this);
    for (int i = int(threadIdx.x); i < AX::Nc; i += NT) lts[i] = lt[i];
  }
  if (PROJ && a.proj_load) {
    if constexpr (PROJ) {
      if (a.src_f64) proj_div_load<T, double, TL, NT, XP>(X, a, l0, n);
      else proj_div_load<T, float, TL, NT, XP>(X, a, l0, n);
    }
  } else if (mode == 1) {
    if (a.src_f64) fast_load(double(0), off_c, xi_c);
    else fast_load(float(0), off_c, xi_c);
  } else if (mode == 2) {
    if (a.src_f64) fast_load(double(0), off_s, xi_s);
    else fast_load(float(0), off_s, xi_s);
  } else {
    if (a.src_f64) generic_load(double(0));
    else generic_load(float(0));
  }
  __syncthreads();

  // ---- forward transform, and optionally eigenvalue division + inverse transform.
  bool mirrored = false;  // the middle step already built the DCT-I input
  if constexpr (KF >= 0) {
    transform_phase<T, NP, NT, PMAX, RADER, SLIM, AX, ST, KF, ZP>(X, Z, ax, a, l0, KF, KB >= 0, KB, mirrored, lts,
                                                                   ctab);
    if constexpr (KB >= 0)
      transform_phase<T, NP, NT, PMAX, RADER, SLIM, AX, ST, KB, ZP>(X, Z, ax, a, l0, KB, false, -1, mirrored, lts,
                                                                     ctab);
  } else {
    const int nphase = a.kind_b >= 0 ? 2 : 1;
    for (int phase = 0; phase < nphase; ++phase) {
      const int kind = phase == 0 ? a.kind_f : a.kind_b;
      transform_phase<T, NP, NT, PMAX, RADER, SLIM, AX, ST, -2, ZP>(X, Z, ax, a, l0, kind,
                                                                     phase == 0 && nphase == 2, a.kind_b, mirrored);
    }
  }

  // ---- store (in update mode the old values are requested first)
  const double shift = (a.update && a.shift) ? a.shift[0] : 0.0;
  auto fast_store = [&](auto off, auto xi) {
    const int tid = opaque_tid();
    if (a.update) {
      char* db = reinterpret_cast<char*>(static_cast<double*>(a.dst) + tbase);
      double old[EF];
#pragma unroll
      for (int e = 0; e < EF; ++e) old[e] = *reinterpret_cast<const double*>(db + off(tid, e) * 8u);
#pragma unroll
      for (int e = 0; e < EF; ++e)
        *reinterpret_cast<double*>(db + off(tid, e) * 8u) = old[e] + double(X[xi(tid, e)]) - shift;
    } else if (a.dst_f64) {
      char* db = reinterpret_cast<char*>(static_cast<double*>(a.dst) + tbase);
#pragma unroll
      for (int e = 0; e < EF; ++e) *reinterpret_cast<double*>(db + off(tid, e) * 8u) = double(X[xi(tid, e)]);
    } else {
      char* db = reinterpret_cast<char*>(static_cast<float*>(a.dst) + tbase);
#pragma unroll
      for (int e = 0; e < EF; ++e) *reinterpret_cast<float*>(db + off(tid, e) * 4u) = float(X[xi(tid, e)]);
    }
  };
  if constexpr (PROJ) {
    if (a.proj_store) {
      if (a.dst_f64) proj_store<T, double, TL, NT, XP>(X, a, l0, n);
      else proj_store<T, float, TL, NT, XP>(X, a, l0, n);
      return;
    }
  }
  if (mode == 1) {
    fast_store(off_c, xi_c);
    return;
  }
  if (mode == 2) {
    fast_store(off_s, xi_s);
    return;
  }
  auto generic_store = [&](auto dst_elem, bool update) {
    using D = decltype(dst_elem);
    const int tid = opaque_tid();
    D* dst = static_cast<D*>(a.dst);
    const int t = tid % TL;
    const int64_t l = l0 + t;
    if (l >= a.nlines) return;
    const int64_t base = (l / a.dst_vnb) * a.dst_va + (l % a.dst_vnb) * a.dst_vb;
    const int64_t sd = a.dst_vd;
    for (int c = 0; c < ELD && c * (NT / TL) < n; c += CH) {
      D old[CH];
      if (update) {
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const int j = tid / TL + (c + i) * (NT / TL);
          old[i] = dst[j < n ? base + int64_t(j) * sd : base];
        }
      }
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        const int j = tid / TL + (c + i) * (NT / TL);
        if (j < n) {
          const T x = X[j * XP + t];
          dst[base + int64_t(j) * sd] = update ? D(double(old[i]) + double(x) - shift) : D(x);
        }
      }
    }
  };
  if (a.update) generic_store(double(0), true);
  else if (a.dst_f64) generic_store(double(0), false);
  else generic_store(float(0), false);
}


// Waves per SIMD the compiler must leave room for: 4 for slim shapes (two
// 512-thread workgroups per CU, at most 128 registers per thread), 2 for
// shapes with the Rader stage and the wide shapes (at most 256 registers, so
// that a second workgroup can hide the first one's global memory latency),
// else 1.
template <int SLIM, int RADER>
struct MinWaves {
  static constexpr int v = SLIM == 1 ? 4 : ((RADER || SLIM == 2) ? 2 : 1);
};

// The batched kernel of a full (non-slim, non-Rader) FP32 shape: held to 128
// registers as well.  Left free it took a few registers more than the
// one-grid kernel (the table reads) and fell to 3 waves per SIMD, one
// 512-thread workgroup per CU.  (The FP64 ones would spill.)
template <typename T, int SLIM, int RADER>
struct MinWavesBatch {
  static constexpr int v = (RADER || SLIM == 2) ? 2 : (SLIM == 1 || sizeof(T) == 4) ? 4 : 1;
};

// One grid: block b owns tile b.
template <typename T, int NP, int NT, int PMAX, int RADER, int SLIM>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MinWaves<SLIM, RADER>::v, 8)))
line_pass(PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  line_pass_body<T, NP, NT, PMAX, RADER, SLIM>(a, xcd_tile(blockIdx.x, gridDim.x), smem);
}

// The same with the projection-step loads and stores.
template <typename T, int NP, int NT, int PMAX, int RADER, int SLIM>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MinWaves<SLIM, RADER>::v, 8)))
line_pass_proj(PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  line_pass_body<T, NP, NT, PMAX, RADER, SLIM, Ax<>, -2, -2, StageList<>, NP, true>(a, xcd_tile(blockIdx.x, gridDim.x),
                                                                                  smem);
}

// Many grids in one launch: block b works on tile tile_idx[b] of grid
// tile_prob[b]; the per-grid pass description comes from a device table and
// the array pointers from per-grid pointer tables.
template <typename T, int NP, int NT, int PMAX, int RADER, int SLIM>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MinWavesBatch<T, SLIM, RADER>::v, 8)))
line_pass_batch(BatchPassArgs b) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int pi = b.tile_prob[blockIdx.x];
  PassArgs a = b.args[pi];
  a.src = b.src_tab[pi];
  a.dst = b.dst_tab[pi];
  a.src_f64 = b.src_f64;
  a.dst_f64 = b.dst_f64;
  a.update = b.update;
  a.shift = (b.update && b.shift_base && a.singular) ? b.shift_base + int64_t(pi) * b.shift_stride : nullptr;
  line_pass_body<T, NP, NT, PMAX, RADER, SLIM>(a, int64_t(b.tile_idx[blockIdx.x]), smem);
}

template <typename T, int NP, int NT, int PMAX, int RADER, int SLIM>
hipError_t launch_lp(const PassArgs& a, hipStream_t s, size_t lds) {
  constexpr int64_t TL = 2 * NP;
  const int64_t blocks = (a.nlines + TL - 1) / TL;
  if (a.proj_load || a.proj_store)
    hipLaunchKernelGGL((line_pass_proj<T, NP, NT, PMAX, RADER, SLIM>), dim3(unsigned(blocks)), dim3(NT), lds, s, a);
  else
    hipLaunchKernelGGL((line_pass<T, NP, NT, PMAX, RADER, SLIM>), dim3(unsigned(blocks)), dim3(NT), lds, s, a);
  return hipGetLastError();
}

template <typename T, int NP, int NT, int PMAX, int RADER, int SLIM>
hipError_t launch_lp_batch(const BatchPassArgs& b, int blocks, hipStream_t s, size_t lds) {
  hipLaunchKernelGGL((line_pass_batch<T, NP, NT, PMAX, RADER, SLIM>), dim3(unsigned(blocks)), dim3(NT), lds, s, b);
  return hipGetLastError();
}

// A kernel specialised for one transform: line length N, DFT length M, work
// length P, kinds KF / KB (KB = -1: no inverse) and the Stockham stage list,
// all compile-time; everything else (arrays, strides, tables, eigenvalues)
// comes from the pass description as in line_pass.
// PAD: complex values of padding per LDS row (pitch NP + PAD): staggers the
// rows that consecutive lanes write in the contiguous-axis load over the
// banks.
template <typename T, int NP, int NT, int RADER, int SLIM, int PAD, int N, int M, int P, int KF, int KB, int... Rs>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MinWaves<SLIM, RADER>::v, 8)))
line_pass_spec(PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  line_pass_body<T, NP, NT, P, RADER, SLIM, Ax<N, M, P>, KF, KB, StageList<Rs...>, NP + PAD>(
      a, xcd_tile(blockIdx.x, gridDim.x), smem);
}

// The same with the projection-step loads and stores (first and last sweeps
// of a projection step; instantiated for the unfused kernels only).
template <typename T, int NP, int NT, int RADER, int SLIM, int PAD, int N, int M, int P, int KF, int KB, int... Rs>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MinWaves<SLIM, RADER>::v, 8)))
line_pass_spec_proj(PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  line_pass_body<T, NP, NT, P, RADER, SLIM, Ax<N, M, P>, KF, KB, StageList<Rs...>, NP + PAD, true>(
      a, xcd_tile(blockIdx.x, gridDim.x), smem);
}

template <typename T, int NP, int NT, int RADER, int SLIM, int PAD, int N, int M, int P, int KF, int KB, int... Rs>
hipError_t launch_spec_t(const PassArgs& a, hipStream_t s, size_t lds) {
  constexpr int64_t TL = 2 * NP;
  if (a.ax.n != N || a.ax.M != M || a.ax.P != P || a.kind_f != KF || a.kind_b != KB ||
      a.ax.nstages != int(sizeof...(Rs)))
    return hipErrorInvalidValue;  // the description must be the one this kernel was compiled for
  const int64_t blocks = (a.nlines + TL - 1) / TL;
  if (a.proj_load || a.proj_store) {
    if constexpr (KB < 0)
      hipLaunchKernelGGL((line_pass_spec_proj<T, NP, NT, RADER, SLIM, PAD, N, M, P, KF, KB, Rs...>),
                         dim3(unsigned(blocks)), dim3(NT), lds, s, a);
    else
      return hipErrorInvalidValue;  // fused kernels carry no projection I/O
  } else {
    hipLaunchKernelGGL((line_pass_spec<T, NP, NT, RADER, SLIM, PAD, N, M, P, KF, KB, Rs...>), dim3(unsigned(blocks)),
                       dim3(NT), lds, s, a);
  }
  return hipGetLastError();
}

template <typename T, int NP, int NT, int RADER, int SLIM, int PAD, int N, int M, int P, int KF, int KB, int... Rs>
hipError_t prepare_spec_t() {
  if constexpr (KB < 0) {
    const hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&line_pass_spec_proj<T, NP, NT, RADER, SLIM, PAD, N, M, P, KF, KB, Rs...>),
        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  return hipFuncSetAttribute(
      reinterpret_cast<const void*>(&line_pass_spec<T, NP, NT, RADER, SLIM, PAD, N, M, P, KF, KB, Rs...>),
      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template <typename T, int NP, int NT, int PMAX, int RADER, int SLIM>
hipError_t prepare_lp() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&line_pass<T, NP, NT, PMAX, RADER, SLIM>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&line_pass_proj<T, NP, NT, PMAX, RADER, SLIM>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&line_pass_batch<T, NP, NT, PMAX, RADER, SLIM>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

}  // namespace mpois
