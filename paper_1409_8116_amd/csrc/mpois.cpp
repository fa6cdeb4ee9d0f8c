// Host side of the solver: argument validation, per-axis transform planning,
// FP64 eigenvalue and twiddle tables, workspace, the launch sequence of one
// solve (Sections 2.1-2.3 of the paper) and the FP64 refinement loop.
#include "mpois.h"

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "tune.h"

namespace mpois {
int num_kernel_cfgs();
void kernel_cfg(int i, int* f64, int* np, int* nt, int* pmax);
int kernel_cfg_rader(int i);
int kernel_cfg_slim(int i);
size_t line_pass_lds(int cfg, int n, int P);
int num_specs();
int find_spec(bool f64, int n, int M, int P, int kind_f, int kind_b, const std::vector<int>& radices);
void spec_shape(int i, int* f64, int* np, int* nt, int* n);
size_t spec_lds(int i);
hipError_t launch_spec(int i, const PassArgs& a, hipStream_t s);
hipError_t prepare_kernels();
hipError_t launch_line_pass(int cfg, const PassArgs& a, hipStream_t s);
int resid_blocks(const int64_t n[3]);
hipError_t launch_resid(const ResidArgs& a, hipStream_t s);
hipError_t launch_finalize(const double* partials, int nblocks, double inv_wsum, double* scalars, hipStream_t s);
hipError_t launch_zero(double* p, int64_t count, hipStream_t s);
hipError_t launch_line_pass_batch(int cfg, const BatchPassArgs& b, int blocks, size_t lds, hipStream_t s);
hipError_t launch_resid_batch(const BatchResidArgs& b, int blocks, hipStream_t s);
hipError_t launch_proj_div(const ProjDev& q, double* g, hipStream_t s);
hipError_t launch_proj_correct(const ProjDev& q, const void* phi, int f64, int mask, int add_p, hipStream_t s);
int find_plane(bool f64, int n, int M, int P, int kind_f, int kind_b, const std::vector<int>& radices);
int num_planes();
void plane_shape(int i, int* f64, int* nt, int* n);
hipError_t launch_plane(int i, const PassArgs& a2, const PassArgs& a1, int inverse, int64_t planes, hipStream_t s);
hipError_t launch_finalize_batch(const double* partials, const int* blk_start, const int* blk_count,
                                 const double* inv_wsum, double* scalars, int count, hipStream_t s);
}  // namespace mpois

using namespace mpois;

namespace {

constexpr int kMaxLds = 160 * 1024;
constexpr int kMaxResidBlocks = 16384;
const int kRadices[] = {8, 4, 2, 3, 5, 7, 11, 13};

// ---------------------------------------------------------------------------- exact angles
// sin / cos of pi * num / den with num reduced modulo 2 den before scaling.
double sinpi_frac(int64_t num, int64_t den) {
  int64_t m = num % (2 * den);
  if (m < 0) m += 2 * den;
  return std::sin(M_PI * double(m) / double(den));
}
double cospi_frac(int64_t num, int64_t den) {
  int64_t m = num % (2 * den);
  if (m < 0) m += 2 * den;
  return std::cos(M_PI * double(m) / double(den));
}

// ---------------------------------------------------------------------------- per-axis math
// An axis's conditions as one code: MPOIS_PERIODIC / MPOIS_DIRICHLET /
// MPOIS_NEUMANN when both faces agree, MPOIS_AXIS_DN (Dirichlet low face,
// Neumann high face) or MPOIS_AXIS_ND otherwise.
int axis_code(int lo, int hi) {
  if (lo == hi) return lo;
  if (lo == MPOIS_DIRICHLET && hi == MPOIS_NEUMANN) return MPOIS_AXIS_DN;
  if (lo == MPOIS_NEUMANN && hi == MPOIS_DIRICHLET) return MPOIS_AXIS_ND;
  return -1;
}

bool mixed_code(int bc) { return bc == MPOIS_AXIS_DN || bc == MPOIS_AXIS_ND; }

// Table 2: forward / backward line transform of an axis.  Mixed faces (not in
// Table 2): the transforms whose basis vectors are sin / cos((k+1/2) pi x/L)
// sampled on the grid -- vertex DST-III / DST-II (Dirichlet low) and
// DCT-III / DCT-II (Neumann low), staggered DST-IV and DCT-IV.
void axis_kinds(int bc, int grid, int* kf, int* kb) {
  if (bc == MPOIS_PERIODIC) { *kf = K_R2HC; *kb = K_HC2R; return; }
  if (bc == MPOIS_AXIS_DN) {
    if (grid == MPOIS_VERTEX) { *kf = K_DST3; *kb = K_DST2; }
    else { *kf = K_DST4; *kb = K_DST4; }
    return;
  }
  if (bc == MPOIS_AXIS_ND) {
    if (grid == MPOIS_VERTEX) { *kf = K_DCT3; *kb = K_DCT2; }
    else { *kf = K_DCT4; *kb = K_DCT4; }
    return;
  }
  if (bc == MPOIS_DIRICHLET) {
    if (grid == MPOIS_VERTEX) { *kf = K_DST1; *kb = K_DST1; }
    else { *kf = K_DST2; *kb = K_DST3; }
    return;
  }
  if (grid == MPOIS_VERTEX) { *kf = K_DCT1; *kb = K_DCT1; }
  else { *kf = K_DCT2; *kb = K_DCT3; }
}

// Complex DFT length used by a line transform of n points.
int64_t axis_dft_length(int kind, int64_t n) {
  if (kind == K_DCT1) return 2 * (n - 1);
  if (kind == K_DST1) return 2 * (n + 1);
  if (kind == K_DST4 || kind == K_DCT4) return 2 * n;
  return n;
}

// Table 2: the factor in front of the backward transform.
double axis_norm(int bc, int grid, int64_t n) {
  if (bc == MPOIS_PERIODIC) return 1.0 / double(n);
  if (mixed_code(bc)) return 1.0 / (2.0 * double(n));
  if (bc == MPOIS_DIRICHLET) return grid == MPOIS_VERTEX ? 1.0 / (2.0 * double(n + 1)) : 1.0 / (2.0 * double(n));
  return grid == MPOIS_VERTEX ? 1.0 / (2.0 * double(n - 1)) : 1.0 / (2.0 * double(n));
}

// Domain length implied by spacing h on the grids of Section 2.1.
double axis_length(int bc, int grid, int64_t n, double h) {
  if (bc == MPOIS_PERIODIC || grid == MPOIS_STAGGERED || mixed_code(bc)) return double(n) * h;
  if (bc == MPOIS_DIRICHLET) return double(n + 1) * h;
  return double(n - 1) * h;
}

// Table 3 (pseudo-spectral) / Table 4 (finite differences), k = 0..n-1.  The
// periodic pseudo-spectral branch uses the aliased wavenumber min(k, n-k).
void axis_eigs(int bc, int grid, int approx, int64_t n, double h, double* out) {
  if (approx == MPOIS_SPECTRAL) {
    const double L = axis_length(bc, grid, n, h);
    for (int64_t k = 0; k < n; ++k) {
      double w;
      if (bc == MPOIS_PERIODIC) w = 2.0 * M_PI * double(std::min(k, n - k)) / L;
      else if (mixed_code(bc)) w = M_PI * (double(k) + 0.5) / L;
      else if (bc == MPOIS_DIRICHLET) w = M_PI * double(k + 1) / L;
      else w = M_PI * double(k) / L;
      out[k] = -w * w;
    }
    return;
  }
  for (int64_t k = 0; k < n; ++k) {
    double s;
    if (bc == MPOIS_PERIODIC) s = sinpi_frac(k, n);
    else if (mixed_code(bc)) s = sinpi_frac(2 * k + 1, 4 * n);
    else if (bc == MPOIS_DIRICHLET) s = grid == MPOIS_VERTEX ? sinpi_frac(k + 1, 2 * (n + 1)) : sinpi_frac(k + 1, 2 * n);
    else s = grid == MPOIS_VERTEX ? sinpi_frac(k, 2 * (n - 1)) : sinpi_frac(k, 2 * n);
    const double v = 2.0 * s / h;
    out[k] = -v * v;
  }
}

// Stockham stages for a DFT of length M: a Rader stage for the prime 73 first
// (only for work lengths up to 1024, where its kernels are instantiated), then
// the odd codelet radices, then the power-of-two part split into as few,
// as even radices as the register budget allows (at most 16 in FP64, 32 in
// FP32).  Returns false if a prime the codelets do not cover remains.
constexpr int kRaderPrime = 73;
bool factor_radices(int64_t M, bool f64, bool exact, std::vector<int>* out, int extra_pow2_stages = 0) {
  out->clear();
  int64_t m = M;
  if (exact && M <= 1024 && m % kRaderPrime == 0) {
    out->push_back(kRaderPrime);
    m /= kRaderPrime;
  }
  // Bluestein lengths are chosen 7-smooth, so they run in every kernel shape
  static const int kOddExact[] = {9, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31};
  static const int kOddSmooth[] = {9, 3, 5, 7};
  const int* odd = exact ? kOddExact : kOddSmooth;
  const int nodd = exact ? 11 : 4;
  for (int oi = 0; oi < nodd; ++oi) {
    const int r = odd[oi];
    while (m % r == 0) {
      out->push_back(r);
      m /= r;
    }
  }
  int e = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++e;
  }
  if (m != 1) return false;
  // after a Rader stage (Rader shapes carry a radix-14 codelet) a lone factor
  // 2 joins a 7: 1022 = 73 x 14 runs in two stages
  if (!out->empty() && out->front() == kRaderPrime && e == 1 && out->back() == 7) {
    out->back() = 14;
    e = 0;
  }
  const int emax = f64 ? 4 : 5;  // radix <= 16 in FP64, <= 32 in FP32 (register budget)
  if (e > 0) {
    int nst = (e + emax - 1) / emax + extra_pow2_stages;
    if (nst > e) nst = e;
    for (int i = 0; i < nst; ++i) {
      const int ei = e / nst + (i < e % nst ? 1 : 0);
      out->push_back(1 << ei);
    }
  }
  return true;
}

// Recursive mixed-radix DFT (sign -1) in FP64 for the Bluestein kernel
// spectrum; lengths factor over the codelet radices.
void host_dft(std::vector<std::complex<double>>& a) {
  const int64_t n = int64_t(a.size());
  if (n <= 1) return;
  int64_t r = 0;
  for (int64_t c : {2, 3, 5, 7, 11, 13})
    if (n % c == 0) { r = c; break; }
  if (r == 0) {  // not reached for planner lengths; direct sum as a safe fallback
    std::vector<std::complex<double>> out(static_cast<size_t>(n));
    for (int64_t k = 0; k < n; ++k)
      for (int64_t j = 0; j < n; ++j)
        out[k] += a[j] * std::complex<double>(cospi_frac(2 * j * k, n), -sinpi_frac(2 * j * k, n));
    a = out;
    return;
  }
  const int64_t m = n / r;
  std::vector<std::vector<std::complex<double>>> sub(static_cast<size_t>(r), std::vector<std::complex<double>>(static_cast<size_t>(m)));
  for (int64_t j = 0; j < m; ++j)
    for (int64_t q = 0; q < r; ++q) sub[q][j] = a[j * r + q];
  for (auto& v : sub) host_dft(v);
  for (int64_t k = 0; k < n; ++k) {
    std::complex<double> acc = 0;
    for (int64_t q = 0; q < r; ++q) acc += sub[q][k % m] * std::complex<double>(cospi_frac(2 * q * k, n), -sinpi_frac(2 * q * k, n));
    a[k] = acc;
  }
}

struct AxisShape {
  int kind_f = 0, kind_b = 0;
  int64_t M = 0, P = 0;
  bool bluestein = false;
  std::vector<int> radices;
  int tag = 0;  // which candidate of axis_variants: 0 default, 1 reversed, 2 one more stage, 3 Bluestein
};

AxisShape plan_axis_shape(int bc, int grid, int64_t n, bool f64) {
  AxisShape s;
  axis_kinds(bc, grid, &s.kind_f, &s.kind_b);
  s.M = axis_dft_length(s.kind_f, n);
  if (factor_radices(s.M, f64, true, &s.radices)) {
    s.P = s.M;
  } else {
    // Bluestein: any cyclic-convolution length >= 2M - 1 works; take the
    // smallest one the codelet radices factor.
    s.bluestein = true;
    s.P = 2 * s.M - 1;
    while (!factor_radices(s.P, f64, false, &s.radices)) ++s.P;
  }
  return s;
}

// Candidate radix plans of one axis for the autotuner, the default first:
// the stage order reversed, the power-of-two part split into one more stage,
// and a Bluestein convolution in place of an exact plan that needs the Rader
// stage or a radix-11/13 codelet.  Deterministic for given arguments (the
// tuner cache stores an index into this list).
std::vector<AxisShape> axis_variants(int bc, int grid, int64_t n, bool f64) {
  std::vector<AxisShape> v;
  const AxisShape d = plan_axis_shape(bc, grid, n, f64);
  v.push_back(d);
  auto add = [&](const AxisShape& s) {
    for (const AxisShape& o : v)
      if (o.bluestein == s.bluestein && o.P == s.P && o.radices == s.radices) return;
    v.push_back(s);
  };
  if (d.radices.size() >= 2) {
    AxisShape r = d;
    std::reverse(r.radices.begin(), r.radices.end());
    r.tag = 1;
    add(r);
  }
  {
    AxisShape x = d;
    x.tag = 2;
    if (factor_radices(d.P, f64, !d.bluestein, &x.radices, 1)) add(x);
  }
  bool big_odd = false;
  for (int r : d.radices) big_odd = big_odd || r == kRaderPrime || ((r & 1) && r >= 11);
  if (!d.bluestein && big_odd && d.M > 1) {
    AxisShape b = d;
    b.bluestein = true;
    b.tag = 3;
    b.P = 2 * d.M - 1;
    while (!factor_radices(b.P, f64, false, &b.radices)) ++b.P;
    add(b);
  }
  return v;
}

bool has_rader(const AxisShape& s) {
  for (int r : s.radices)
    if (r == kRaderPrime) return true;
  return false;
}

// Odd radices above 9 the plan needs: 0 none, 1 radix 11 or 13 (codelets in
// the full and the wide shapes, not in the slim ones), 2 a prime 17..31
// (codelets in the wide shapes only).
int odd_class(const AxisShape& s) {
  int c = 0;
  for (int r : s.radices)
    if ((r & 1) && r >= 11 && r != kRaderPrime) c = std::max(c, r >= 17 ? 2 : 1);
  return c;
}

// ---------------------------------------------------------------------------- device tables
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool pooled = false;  // carved from the plan's table pool (freed with the pool)
};

struct AxisTables {
  AxisShape shape;
  int64_t n = 0;
  DevBuf tw, pre, chirp, bhat, cs, stages;
  AxisDev dev{};
};

template <typename T>
void to_prec(const std::vector<std::complex<double>>& src, std::vector<T>* dst) {
  dst->resize(src.size() * 2);
  for (size_t i = 0; i < src.size(); ++i) {
    (*dst)[2 * i] = T(src[i].real());
    (*dst)[2 * i + 1] = T(src[i].imag());
  }
}

// ---------------------------------------------------------------------------- plan
struct Pass {
  PassArgs args{};
  int cfg = 0;    // generic kernel shape (cfgs.h); batches always use it
  int spec = -1;  // specialised kernel (specs.h) used by single-grid executes, or -1
  int axis = 0;   // axis this pass transforms
  int table = -1; // index of its axis tables in the plan
};

// Kernel ids reported by mpois_profile: generic shapes 0.., residual 100,
// reduction 101, specialised kernels kSpecBase + spec index.
constexpr int kSpecBase = 200;
constexpr int kPlaneBase = 300;  // plane kernels (planes.h)

struct SubPlan {
  int ndim = 0;
  int64_t n[3] = {1, 1, 1};     // padded to 3D: leading unit dims
  int64_t npts = 0;
  int bc[3] = {0, 0, 0}, grid[3] = {0, 0, 0};  // bc: axis codes (axis_code)
  int face[3][2] = {{0, 0}, {0, 0}, {0, 0}};     // conditions of the low / high face
  double h[3] = {1, 1, 1};
  bool singular = false;
  double wsum = 0;              // sum of gauge weights
  std::vector<DevBuf> lam;      // scaled eigenvalues per axis (working precision)
  std::vector<Pass> passes;     // forward ... fused ... inverse
  ResidArgs resid{};
  int rperm[3] = {0, 1, 2};     // residual axis e is padded axis rperm[e]
  int plane = -1;               // plane kernel for the last two axes of a 3D grid, or -1
};

// Per-launch record of a profiled execute.
struct ProfRec {
  int kernel;      // line-pass configuration index, or 100 residual, 101 finalisation
  double bytes;    // algorithmic HBM bytes of the launch
  hipEvent_t end;  // recorded after the launch
};

// Batched execution: per pass index, one launch per kernel shape over all
// grids that use it; per-grid descriptions in device tables.
struct BatchGroup {
  int cfg = 0;
  int blocks = 0;
  size_t lds = 0;
  DevBuf tile_prob, tile_idx;
};

struct BatchPass {
  DevBuf args;  // PassArgs per grid
  std::vector<BatchGroup> groups;
};

struct BatchState {
  std::vector<BatchPass> passes;
  DevBuf rhs_tab, phi_tab, work_tab;  // per-grid device pointers
  DevBuf resid_args, blk_prob, blk_start, blk_count, inv_wsum, partials;
  int resid_blocks = 0;
  bool any_singular = false;
  // Pointer tables as last validated and uploaded: pinned host staging
  // (rhs pointers, then phi pointers), and an event that marks the end of the
  // upload so the staging is not rewritten while a copy from it is pending.
  void** staging = nullptr;
  hipEvent_t uploaded = nullptr;
  bool have_tables = false;
  // The kernel-shape groups of one sweep touch disjoint grids: they run on
  // the execute's stream and side streams (forked and joined by events), so
  // a small group fills the chip while a large one drains.
  std::vector<hipStream_t> side;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
};

struct Graph {
  const void* rhs = nullptr;
  void* phi = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // namespace

struct mpois_plan_s {
  int approx = 0, prec = 0, max_iter = 1;
  double rtol = 0;
  unsigned flags = 0;
  int device = 0;
  bool f64work = true;
  std::vector<AxisTables> tables;
  std::map<std::string, int> table_index;  // shape_key -> index into tables
  std::vector<SubPlan> subs;
  DevBuf work;       // FP32 working array (refinement)
  DevBuf partials;   // resid partials
  DevBuf scalars;    // S_COUNT doubles per grid
  DevBuf proj_g;     // FP64 divergence of a projection step (refinement plans, first call)
  size_t bytes = 0;
  const void* last_rhs = nullptr;
  void* last_phi = nullptr;
  const void* checked_rhs = nullptr;  // last pointer pair that passed check_ptrs
  void* checked_phi = nullptr;
  int64_t last_rhs_view[3] = {0, 0, 0};  // padded strides of the last execute's arrays
  int64_t last_phi_view[3] = {0, 0, 0};
  bool last_view = false;                 // the last execute used views
  std::vector<const void*> last_rhs_b;
  std::vector<void*> last_phi_b;
  int last_iters = 0;
  Graph graph;
  hipStream_t cap_stream = nullptr;
  hipEvent_t prof_start = nullptr;
  BatchState batch;
  bool batched = false;
  std::vector<ProfRec> prof;
  size_t prof_used = 0;
  bool profiling = false;
  TuneSession* tune = nullptr;  // measurement scratch while the plan is built
  std::vector<void*> pool;      // chunks holding the small device buffers
  size_t pool_used = 0;         // bytes used in the last chunk
};

namespace {

// Named ranges (roctx) around the library's calls and the phases of a solve,
// for rocprofv3 --marker-trace, when the environment sets MPOIS_TRACE=1
// (read on every call, so a process can switch it).
struct TraceRange {
  bool on;
  explicit TraceRange(const char* name) {
    const char* e = std::getenv("MPOIS_TRACE");
    on = e && e[0] == '1';
    if (on) roctxRangePushA(name);
  }
  ~TraceRange() {
    if (on) roctxRangePop();
  }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

bool fault_alloc() {
  const char* e = std::getenv("MPOIS_FAULT_ALLOC");
  return e && e[0] == '1';
}

// Small buffers (tables, descriptions) are carved from pool chunks of
// kPoolChunk bytes, so a plan with thousands of axis tables makes few
// device allocations.
constexpr size_t kPoolChunk = size_t(8) << 20;
constexpr size_t kPoolMax = size_t(1) << 20;

mpois_status dev_alloc(mpois_plan_s* pl, DevBuf* b, size_t bytes) {
  if (bytes == 0) return MPOIS_OK;
  if (fault_alloc()) return MPOIS_ERR_NOMEM;
  if (bytes <= kPoolMax) {
    const size_t need = (bytes + 255) & ~size_t(255);
    if (pl->pool.empty() || pl->pool_used + need > kPoolChunk) {
      void* c = nullptr;
      if (hipMalloc(&c, kPoolChunk) != hipSuccess) {
        (void)hipGetLastError();
        return MPOIS_ERR_NOMEM;
      }
      pl->pool.push_back(c);
      pl->pool_used = 0;
      pl->bytes += kPoolChunk;
    }
    b->p = static_cast<char*>(pl->pool.back()) + pl->pool_used;
    b->bytes = bytes;
    b->pooled = true;
    pl->pool_used += need;
    return MPOIS_OK;
  }
  if (hipMalloc(&b->p, bytes) != hipSuccess) {
    b->p = nullptr;
    (void)hipGetLastError();
    return MPOIS_ERR_NOMEM;
  }
  b->bytes = bytes;
  pl->bytes += bytes;
  return MPOIS_OK;
}

template <typename V>
mpois_status dev_upload(mpois_plan_s* pl, DevBuf* b, const std::vector<V>& host) {
  if (host.empty()) return MPOIS_OK;
  mpois_status st = dev_alloc(pl, b, host.size() * sizeof(V));
  if (st != MPOIS_OK) return st;
  if (hipMemcpy(b->p, host.data(), b->bytes, hipMemcpyHostToDevice) != hipSuccess) return MPOIS_ERR_DEVICE;
  return MPOIS_OK;
}

void dev_free(DevBuf* b) {
  if (b->p && !b->pooled) (void)hipFree(b->p);
  b->p = nullptr;
  b->bytes = 0;
}

template <typename T>
mpois_status build_axis_tables(mpois_plan_s* pl, AxisTables* at) {
  const AxisShape& s = at->shape;
  const int64_t n = at->n;
  // Stockham stages and their twiddles e^{-2 pi i r k/(ns R)}.
  std::vector<std::complex<double>> tw, cs;
  AxisDev& d = at->dev;
  d.n = int(n);
  d.M = int(s.M);
  d.P = int(s.P);
  d.bluestein = s.bluestein ? 1 : 0;
  d.nstages = int(s.radices.size());
  std::vector<Stage> stages(s.radices.size() + 1);
  int64_t ns = 1;
  for (size_t i = 0; i < s.radices.size(); ++i) {
    const int R = s.radices[i];
    Stage& st = stages[i];
    st.radix = R;
    st.ns = int(ns);
    // q = umulhi(b, ns_mul) equals b / ns for b < 2^16 and ns < 2^16 (the
    // error b 2^-32 of the scaled reciprocal stays below 1/ns)
    st.ns_mul = ns > 1 ? unsigned((uint64_t(1) << 32) / uint64_t(ns) + 1) : 0u;
    st.tw_off = int(tw.size());
    for (int64_t k = 0; k < ns; ++k)
      for (int r = 1; r < R; ++r) {
        const int64_t num = 2 * int64_t(r) * k, den = ns * R;
        tw.emplace_back(cospi_frac(num, den), -sinpi_frac(num, den));
      }
    st.cs_off = int(cs.size());
    if (R == kRaderPrime) {
      // Rader kernel spectrum: dhat = DFT_{R-1}(d) / (R-1), d_j = e^{-2 pi i g^{-j} / R}
      const int L = R - 1;
      int g = 2;
      for (; g < R; ++g) {  // smallest primitive root
        int64_t x = 1;
        int order = 0;
        do {
          x = x * g % R;
          ++order;
        } while (x != 1);
        if (order == L) break;
      }
      int64_t ginv = 1;
      for (int e = 0; e < R - 2; ++e) ginv = ginv * g % R;
      std::vector<std::complex<double>> d(static_cast<size_t>(L));
      int64_t gp = 1;
      for (int j = 0; j < L; ++j) {
        d[j] = {cospi_frac(2 * gp, R), -sinpi_frac(2 * gp, R)};
        gp = gp * ginv % R;
      }
      host_dft(d);
      for (auto& x : d) cs.push_back(x / double(L));
      // twiddles e^{-2 pi i j / L} of the two-level length-L DFT
      for (int j = 0; j < L; ++j) cs.emplace_back(cospi_frac(2 * j, L), -sinpi_frac(2 * j, L));
      // the same constants in lane order for G = 2 and G = 4 lanes per
      // butterfly (entry k1 G + s): dhat[k1 + K bitrev(s)], then the twiddle
      // e^{-2 pi i s k1 / L}; the kernels stage one block in LDS
      const size_t d0 = cs.size() - size_t(2 * L);  // dhat, just written
      for (int G : {2, 4}) {
        const int K = L / G;
        auto bitrev = [G](int x) { return G == 2 ? x : ((x & 1) << 1) | (x >> 1); };
        for (int k1 = 0; k1 < K; ++k1)
          for (int sl = 0; sl < G; ++sl) cs.push_back(cs[d0 + k1 + K * bitrev(sl)]);
        for (int k1 = 0; k1 < K; ++k1)
          for (int sl = 0; sl < G; ++sl) cs.emplace_back(cospi_frac(2 * sl * k1, L), -sinpi_frac(2 * sl * k1, L));
      }
    }
    ns *= R;
  }
  if (tw.empty()) tw.emplace_back(1.0, 0.0);
  if (cs.empty()) cs.emplace_back(1.0, 0.0);
  mpois_status st = dev_upload(pl, &at->stages, stages);
  if (st != MPOIS_OK) return st;
  std::vector<T> h;
  to_prec(tw, &h);
  if ((st = dev_upload(pl, &at->tw, h)) != MPOIS_OK) return st;
  to_prec(cs, &h);
  if ((st = dev_upload(pl, &at->cs, h)) != MPOIS_OK) return st;
  // e^{-i pi k/(2n)} for the DCT-II/III, DST-II/III and type-IV kinds, then
  // e^{-i pi/(4n)} (the type-IV post-twiddle's half step)
  auto uses_pre = [](int k) {
    return k == K_DCT2 || k == K_DCT3 || k == K_DST2 || k == K_DST3 || k == K_DST4 || k == K_DCT4;
  };
  if (uses_pre(s.kind_f) || uses_pre(s.kind_b)) {
    std::vector<std::complex<double>> pre(static_cast<size_t>(n + 1));
    for (int64_t k = 0; k < n; ++k) pre[k] = {cospi_frac(k, 2 * n), -sinpi_frac(k, 2 * n)};
    pre[n] = {cospi_frac(1, 4 * n), -sinpi_frac(1, 4 * n)};
    to_prec(pre, &h);
    if ((st = dev_upload(pl, &at->pre, h)) != MPOIS_OK) return st;
  }
  // Bluestein: chirp w_m = e^{-i pi m^2/M}, kernel b = conj(w) wrapped, its DFT / P.
  if (s.bluestein) {
    std::vector<std::complex<double>> w(static_cast<size_t>(s.M)), b(size_t(s.P), {0.0, 0.0});
    for (int64_t m = 0; m < s.M; ++m) {
      const int64_t q = (m * m) % (2 * s.M);
      w[m] = {cospi_frac(q, s.M), -sinpi_frac(q, s.M)};
    }
    for (int64_t m = 0; m < s.M; ++m) b[m] = std::conj(w[m]);
    for (int64_t m = 1; m < s.M; ++m) b[s.P - m] = std::conj(w[m]);
    host_dft(b);
    for (auto& x : b) x /= double(s.P);
    to_prec(w, &h);
    if ((st = dev_upload(pl, &at->chirp, h)) != MPOIS_OK) return st;
    to_prec(b, &h);
    if ((st = dev_upload(pl, &at->bhat, h)) != MPOIS_OK) return st;
  }
  d.st = static_cast<const Stage*>(at->stages.p);
  d.tw = at->tw.p;
  d.cs = at->cs.p;
  d.pre = at->pre.p;
  d.chirp = at->chirp.p;
  d.bhat = at->bhat.p;
  return MPOIS_OK;
}

// Kernel configuration for a line pass.  Candidates: shapes of the working
// precision that hold the work length in LDS and have the codelets the stage
// list needs (the Rader stage only in RADER shapes; radix 11/13 only in
// non-slim shapes, primes 17..31 only in the wide shapes).  Preference: slim shapes that fit two workgroups per CU
// (LDS <= 80 KB), then the widest tile; with a Rader stage, 256 threads and
// the narrowest tile.  MPOIS_FLAG_TUNE replaces this guess
// by a measurement.
bool cfg_fits(int i, bool f64, int n, int P, bool rader, int odd) {
  int cf64, np, nt, pmax;
  kernel_cfg(i, &cf64, &np, &nt, &pmax);
  if ((cf64 != 0) != f64 || P > pmax) return false;
  if (rader && !kernel_cfg_rader(i)) return false;
  if (odd >= 1 && kernel_cfg_slim(i) == 1) return false;
  if (odd == 2 && kernel_cfg_slim(i) != 2) return false;
  return line_pass_lds(i, n, P) <= size_t(kMaxLds);
}

int default_cfg(bool f64, int n, int P, bool rader, int odd) {
  int best = -1;
  long best_score = -1;
  for (int i = 0; i < num_kernel_cfgs(); ++i) {
    if (!cfg_fits(i, f64, n, P, rader, odd)) continue;
    int cf64, np, nt, pmax;
    kernel_cfg(i, &cf64, &np, &nt, &pmax);
    const bool two = kernel_cfg_slim(i) == 1 && line_pass_lds(i, n, P) <= size_t(kMaxLds / 2);
    // a Rader stage keeps many values per lane: smaller workgroups and tiles
    // leave the registers to it (measured fastest on 512^3 DCT-I passes)
    // ties go to the smaller work-length bound (fewer guarded unrolled steps)
    const long score = (rader ? (nt == 256 ? 10000 : 0) - np * 100 : (two ? 10000 : 0) + np * 100 + (nt == 512 ? 10 : 0)) -
                       pmax / 1024;
    if (score > best_score) {
      best = i;
      best_score = score;
    }
  }
  return best;
}

// Closure of one end of an axis from that face's condition.  A vertex axis of
// one unknown with a Neumann face and a Dirichlet face mirrors the Dirichlet
// node, so both ends see 0.
int closure_of(int face, int grid) {
  if (face == MPOIS_PERIODIC) return C_PER;
  if (face == MPOIS_DIRICHLET) return grid == MPOIS_VERTEX ? C_DV : C_DS;
  return grid == MPOIS_VERTEX ? C_NV : C_NS;
}

void axis_closures(int lo, int hi, int grid, int64_t n, int* clo, int* chi) {
  *clo = closure_of(lo, grid);
  *chi = closure_of(hi, grid);
  if (lo != hi && grid == MPOIS_VERTEX && n == 1) *clo = *chi = C_DV;
}

mpois_status validate_one(const mpois_grid_desc* g, int approx, int prec, int max_iter) {
  if (!g) return MPOIS_ERR_INVALID;
  if (g->ndim < 1 || g->ndim > 3) return MPOIS_ERR_INVALID;
  if (approx != MPOIS_SPECTRAL && approx != MPOIS_FD2) return MPOIS_ERR_INVALID;
  if (prec != MPOIS_F64 && prec != MPOIS_F32 && prec != MPOIS_F32_REFINE) return MPOIS_ERR_INVALID;
  int64_t total = 1;
  for (int d = 0; d < g->ndim; ++d) {
    const int b0 = g->bc[d][0], b1 = g->bc[d][1];
    if (b0 < 0 || b0 > 2 || b1 < 0 || b1 > 2) return MPOIS_ERR_INVALID;
    if ((b0 == MPOIS_PERIODIC) != (b1 == MPOIS_PERIODIC)) return MPOIS_ERR_INVALID;
    if (g->grid[d] != MPOIS_VERTEX && g->grid[d] != MPOIS_STAGGERED) return MPOIS_ERR_INVALID;
    if (!(std::isfinite(g->h[d]) && g->h[d] > 0)) return MPOIS_ERR_INVALID;
    if (g->n[d] < 1) return MPOIS_ERR_INVALID;
    if (b0 == MPOIS_NEUMANN && b1 == MPOIS_NEUMANN && g->grid[d] == MPOIS_VERTEX && g->n[d] < 2)
      return MPOIS_ERR_INVALID;
    if (g->n[d] > (1 << 20)) return MPOIS_ERR_UNSUPPORTED;
    total *= g->n[d];
    if (total > (int64_t(1) << 34)) return MPOIS_ERR_UNSUPPORTED;
  }
  if (!(std::isfinite(g->shift) && g->shift >= 0.0)) return MPOIS_ERR_INVALID;
  if (prec == MPOIS_F32_REFINE) {
    if (approx == MPOIS_SPECTRAL) return MPOIS_ERR_UNSUPPORTED;
    if (max_iter < 1 || max_iter > 64) return MPOIS_ERR_INVALID;
  }
  // every axis must fit one of the kernel shapes
  for (int d = 0; d < g->ndim; ++d) {
    AxisShape s = plan_axis_shape(axis_code(g->bc[d][0], g->bc[d][1]), g->grid[d], g->n[d], prec == MPOIS_F64);
    if (default_cfg(prec == MPOIS_F64, int(g->n[d]), int(s.P), has_rader(s), odd_class(s)) < 0)
      return MPOIS_ERR_UNSUPPORTED;
  }
  return MPOIS_OK;
}

mpois_status device_ready(int* dev) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    (void)hipGetLastError();
    return MPOIS_ERR_DEVICE;
  }
  if (hipGetDevice(dev) != hipSuccess) return MPOIS_ERR_DEVICE;
  static bool prepared = false;
  if (!prepared) {
    if (prepare_kernels() != hipSuccess) return MPOIS_ERR_DEVICE;
    prepared = true;
  }
  return MPOIS_OK;
}

template <typename T>
mpois_status upload_lam(mpois_plan_s* pl, DevBuf* b, const std::vector<double>& lam) {
  std::vector<T> h(lam.size());
  for (size_t i = 0; i < lam.size(); ++i) h[i] = T(lam[i]);
  return dev_upload(pl, b, h);
}

std::string shape_key(int bc, int grid, int64_t n, const AxisShape& sh) {
  std::string k = std::to_string(bc * 2 + (bc == MPOIS_PERIODIC ? 0 : grid)) + "/" + std::to_string(sh.kind_f) + "." +
                  std::to_string(sh.kind_b) + "/" + std::to_string(n) + "/" +
                  std::to_string(sh.P) + (sh.bluestein ? "b" : "e");
  for (int r : sh.radices) k += "." + std::to_string(r);
  return k;
}

// Device tables of one axis transform with radix plan `shape`, shared by
// every pass of the plan that uses the same one.
int table_for(mpois_plan_s* pl, int bc, int grid, int64_t n, const AxisShape& shape, mpois_status* st) {
  const std::string key = shape_key(bc, grid, n, shape);
  auto it = pl->table_index.find(key);
  if (it != pl->table_index.end()) return it->second;
  AxisTables at;
  at.shape = shape;
  at.n = n;
  pl->tables.push_back(at);
  const int idx = int(pl->tables.size()) - 1;
  *st = pl->f64work ? build_axis_tables<double>(pl, &pl->tables[idx]) : build_axis_tables<float>(pl, &pl->tables[idx]);
  pl->table_index[key] = idx;
  return idx;
}

// Measured choice of radix plan and kernel shape for one pass (MPOIS_FLAG_TUNE).
// Candidates: every radix plan of axis_variants times every kernel shape that
// holds it, each timed on scratch arrays.  Single-grid plans time the pass's
// own line count and cache the decision per (precision, kinds, axis kind,
// length, stride class, line count).  Batch plans share the chip with the
// other grids, so per-line throughput at full occupancy is what counts: each
// candidate runs at least 2048 workgroups' worth of lines, and the decision
// (a variant tag and a shape) is made once per bucket of similar passes --
// precision, kinds, axis kind, stride class, radix family (Rader, radix
// 11/13, Bluestein or smooth) and the power-of-two size class of the work
// length -- from its first member, then reused by the others.  Returns the
// index of the chosen plan's tables (and the shape in *cfg), or -1 if
// nothing could be measured.
int tune_axis_pass(mpois_plan_s* pl, const PassArgs& proto, int bc, int grid, int64_t n, int* cfg,
                   mpois_status* st) {
  const bool f64 = pl->f64work;
  const bool batch = pl->subs.size() > 1;
  const std::vector<AxisShape> vars = axis_variants(bc, grid, n, f64);
  const AxisShape& d0 = vars[0];
  std::string key = std::string(f64 ? "f64" : "f32") + "/kf" + std::to_string(proto.kind_f) + "/kb" +
                    std::to_string(proto.kind_b) + "/bc" + std::to_string(bc) + std::to_string(grid) +
                    (proto.inner == 1 ? "/c" : "/s");
  if (batch) {
    int pc = 0;
    while ((int64_t(1) << pc) < d0.P) ++pc;
    const char* fam = has_rader(d0) ? "r" : odd_class(d0) ? "o" : d0.bluestein ? "b" : "s";
    key += std::string("/tput/") + fam + std::to_string(pc) + "/";
    // and how many workgroups of each shape fit a CU (LDS) at this length:
    // members of a bucket then see the same occupancy per shape
    for (int c = 0; c < num_kernel_cfgs(); ++c) {
      const bool fits = cfg_fits(c, f64, int(n), int(d0.P), has_rader(d0), odd_class(d0));
      const size_t lds = line_pass_lds(c, int(n), int(d0.P));
      key += fits ? char('0' + std::min<size_t>(4, size_t(kMaxLds) * 2 / std::max<size_t>(lds, 1) / 2)) : '-';
    }
  } else {
    key += "/n" + std::to_string(n) + "/l" + std::to_string(proto.nlines);
  }
  // MPOIS_TUNE_VARIANT=k restricts the candidates to radix plan k of
  // axis_variants (when it exists), bypassing the cache: a test hook that
  // makes every plan variant reachable.
  const char* force = std::getenv("MPOIS_TUNE_VARIANT");
  const int only = force ? std::atoi(force) : -1;
  int tag = -1, ci = -1;
  if (only < 0 && tune_lookup(key, &tag, &ci)) {
    // the variant with the stored tag (else the default) and the stored shape
    // when it holds this length (else the default shape)
    size_t v = 0;
    for (size_t i = 0; i < vars.size(); ++i)
      if (vars[i].tag == tag) v = i;
    const AxisShape& sh = vars[v];
    const bool fits = ci >= 0 && cfg_fits(ci, f64, int(n), int(sh.P), has_rader(sh), odd_class(sh));
    *cfg = fits ? ci : default_cfg(f64, int(n), int(sh.P), has_rader(sh), odd_class(sh));
    if (*cfg < 0) return -1;
    return table_for(pl, bc, grid, n, sh, st);
  }
  if (!pl->tune) pl->tune = tune_begin();
  double best = 1e300;
  int best_t = -1, best_tag = -1;
  ci = -1;
  for (size_t v = 0; v < vars.size(); ++v) {
    if (only >= 0 && only < int(vars.size()) && int(v) != only) continue;
    const AxisShape& sh = vars[v];
    const int t = table_for(pl, bc, grid, n, sh, st);
    if (*st != MPOIS_OK) return -1;
    PassArgs a = proto;
    a.ax = pl->tables[t].dev;
    for (int c = 0; c < num_kernel_cfgs(); ++c) {
      if (!cfg_fits(c, f64, int(n), int(sh.P), has_rader(sh), odd_class(sh))) continue;
      int cf64, np, nt, pmax;
      kernel_cfg(c, &cf64, &np, &nt, &pmax);
      int64_t lines = proto.nlines;
      if (batch) {
        lines = std::max<int64_t>(lines, int64_t(2048) * 2 * np);
        lines = (lines + proto.inner - 1) / proto.inner * proto.inner;
      }
      const double ms = batch ? tune_time_batch(pl->tune, a, c, lines) : tune_time(pl->tune, a, c, lines);
      const double per_line = ms / double(lines);
      if (std::getenv("MPOIS_LOG"))
        std::fprintf(stderr, "[mpois tune] %s n%lld plan %zu shape %d: %.4f ms over %lld lines\n", key.c_str(),
                     static_cast<long long>(n), v, c, ms, static_cast<long long>(lines));
      if (ms >= 0 && per_line < best) {
        best = per_line;
        best_t = t;
        best_tag = sh.tag;
        ci = c;
      }
    }
  }
  if (best_t < 0) return -1;
  if (std::getenv("MPOIS_LOG"))
    std::fprintf(stderr, "[mpois tune] %s n%lld -> plan tag %d shape %d (untuned shape %d)\n", key.c_str(),
                 static_cast<long long>(n), best_tag, ci,
                 default_cfg(f64, int(n), int(d0.P), has_rader(d0), odd_class(d0)));
  if (only < 0) tune_store(key, best_tag, ci);
  *cfg = ci;
  return best_t;
}

mpois_status build_sub(mpois_plan_s* pl, const mpois_grid_desc* g, SubPlan* sp) {
  const int D = g->ndim;
  sp->ndim = D;
  // pad to 3D with leading unit axes
  for (int d = 0; d < D; ++d) {
    const int e = 3 - D + d;
    sp->n[e] = g->n[d];
    sp->h[e] = g->h[d];
    sp->bc[e] = axis_code(g->bc[d][0], g->bc[d][1]);
    sp->face[e][0] = g->bc[d][0];
    sp->face[e][1] = g->bc[d][1];
    sp->grid[e] = g->bc[d][0] == MPOIS_PERIODIC ? MPOIS_VERTEX : g->grid[d];
  }
  sp->npts = sp->n[0] * sp->n[1] * sp->n[2];
  // singular: no shift and every axis periodic or Neumann on both faces
  sp->singular = g->shift == 0.0;
  for (int d = 0; d < D; ++d) {
    const int code = axis_code(g->bc[d][0], g->bc[d][1]);
    if (code != MPOIS_PERIODIC && code != MPOIS_NEUMANN) sp->singular = false;
  }
  // weights sum
  double wsum = 1.0;
  for (int d = 0; d < D; ++d) {
    const int64_t n = g->n[d];
    wsum *= (g->bc[d][0] == MPOIS_NEUMANN && g->bc[d][1] == MPOIS_NEUMANN && g->grid[d] == MPOIS_VERTEX)
                ? double(n - 1)
                : double(n);
  }
  sp->wsum = wsum;
  // tables, eigenvalues scaled by the product of the backward normalisations
  double c = 1.0;
  for (int d = 0; d < D; ++d) c *= axis_norm(axis_code(g->bc[d][0], g->bc[d][1]), g->grid[d], g->n[d]);
  mpois_status st = MPOIS_OK;
  sp->lam.resize(D);
  for (int d = 0; d < D; ++d) {
    std::vector<double> lam(static_cast<size_t>(g->n[d]));
    axis_eigs(axis_code(g->bc[d][0], g->bc[d][1]), g->grid[d], pl->approx, g->n[d], g->h[d], lam.data());
    // the Helmholtz shift joins the divisor through axis 0's table, which
    // every divisor contains: (sum_d lambda_d - sigma) / c
    if (d == 0)
      for (auto& v : lam) v -= g->shift;
    for (auto& v : lam) v /= c;
    st = pl->f64work ? upload_lam<double>(pl, &sp->lam[d], lam) : upload_lam<float>(pl, &sp->lam[d], lam);
    if (st != MPOIS_OK) return st;
  }
  // passes (input and output pointers are filled at execute time)
  auto axis_pass = [&](int d, bool fused, bool inverse) {
    Pass p;
    const int bc = axis_code(g->bc[d][0], g->bc[d][1]), grd = g->grid[d];
    const int64_t n = g->n[d];
    const AxisShape shape = plan_axis_shape(bc, grd, n, pl->f64work);
    PassArgs& a = p.args;
    int64_t inner = 1;
    for (int e = d + 1; e < D; ++e) inner *= g->n[e];
    a.nlines = 1;
    for (int e = 0; e < D; ++e)
      if (e != d) a.nlines *= g->n[e];
    a.inner = inner;
    a.kind_f = inverse ? shape.kind_b : shape.kind_f;
    a.kind_b = fused ? shape.kind_b : -1;
    a.singular = sp->singular ? 1 : 0;
    if (fused) {
      a.lam_this = sp->lam[d].p;
      if (D >= 2) a.lam_a = sp->lam[1].p;
      if (D == 3) {
        a.lam_b = sp->lam[2].p;
        a.nb = g->n[2];
      }
    }
    p.axis = d;
    int ti = -1;
    if (tune_enabled(pl->flags)) {
      ti = tune_axis_pass(pl, a, bc, grd, n, &p.cfg, &st);
      if (st != MPOIS_OK) return p;
    }
    if (ti < 0) {
      ti = table_for(pl, bc, grd, n, shape, &st);
      if (st != MPOIS_OK) return p;
      p.cfg = default_cfg(pl->f64work, int(n), int(shape.P), has_rader(shape), odd_class(shape));
    }
    a.ax = pl->tables[ti].dev;
    p.table = ti;
    // C-contiguous addressing of src and dst (views override it per execute)
    a.src_vnb = a.dst_vnb = inner;
    a.src_va = a.dst_va = n * inner;
    a.src_vb = a.dst_vb = 1;
    a.src_vd = a.dst_vd = inner;
    a.contig = 1;
    // a kernel compiled for exactly this transform, unless switched off
    // (MPOIS_NO_SPEC=1, a test hook comparing it with the generic shapes)
    const char* nospec = std::getenv("MPOIS_NO_SPEC");
    if (!(nospec && nospec[0] == '1')) {
      const AxisShape& sh = pl->tables[ti].shape;
      p.spec = find_spec(pl->f64work, int(n), int(sh.M), int(sh.P), a.kind_f, a.kind_b, sh.radices);
      if (p.spec >= 0 && spec_lds(p.spec) > size_t(kMaxLds)) p.spec = -1;
    }
    return p;
  };
  for (int d = D - 1; d >= 1 && st == MPOIS_OK; --d) sp->passes.push_back(axis_pass(d, false, false));
  if (st == MPOIS_OK) sp->passes.push_back(axis_pass(0, true, false));
  for (int d = 1; d < D && st == MPOIS_OK; ++d) sp->passes.push_back(axis_pass(d, false, true));
  if (st != MPOIS_OK) return st;
  for (const Pass& p : sp->passes)
    if (p.cfg < 0) return MPOIS_ERR_UNSUPPORTED;
  // both of the last two axes of a 3D grid in one plane sweep, when they share
  // a transform a plane kernel is compiled for (MPOIS_NO_PLANE=1: never, a
  // test hook comparing it with the per-axis sweeps)
  const char* noplane = std::getenv("MPOIS_NO_PLANE");
  if (D == 3 && !(noplane && noplane[0] == '1')) {
    const AxisShape& s2 = pl->tables[sp->passes[0].table].shape;
    const AxisShape& s1 = pl->tables[sp->passes[1].table].shape;
    // one set of tables (the plane kernel stages one twiddle table for both)
    if (sp->passes[0].table == sp->passes[1].table && sp->passes[3].table == sp->passes[4].table &&
        g->n[1] == g->n[2] && s1.kind_f == s2.kind_f && s1.kind_b == s2.kind_b && !s2.bluestein)
      sp->plane = find_plane(pl->f64work, int(g->n[2]), int(s2.M), int(s2.P), s2.kind_f, s2.kind_b, s2.radices);
  }
  // residual description
  ResidArgs& r = sp->resid;
  for (int e = 0; e < 3; ++e) {
    r.n[e] = sp->n[e];
    r.ps[e] = r.gs[e] = (e == 0 ? sp->n[1] * sp->n[2] : e == 1 ? sp->n[2] : 1);
    const bool real_axis = e >= 3 - D;
    r.clo[e] = r.chi[e] = C_NONE;
    if (real_axis) axis_closures(sp->face[e][0], sp->face[e][1], sp->grid[e], sp->n[e], &r.clo[e], &r.chi[e]);
    r.inv_h2[e] = real_axis ? 1.0 / (sp->h[e] * sp->h[e]) : 0.0;
  }
  r.shift = g->shift;
  if (D == 2) {
    // the residual kernel marches along its axis 0 with the neighbours in
    // registers: give it the grid's first axis rather than the unit one
    std::swap(r.n[0], r.n[1]);
    std::swap(r.ps[0], r.ps[1]);
    std::swap(r.gs[0], r.gs[1]);
    std::swap(r.clo[0], r.clo[1]);
    std::swap(r.chi[0], r.chi[1]);
    std::swap(r.inv_h2[0], r.inv_h2[1]);
    sp->rperm[0] = 1;
    sp->rperm[1] = 0;
  }
  return MPOIS_OK;
}

void free_plan(mpois_plan_s* pl) {
  for (auto& t : pl->tables) {
    dev_free(&t.tw);
    dev_free(&t.pre);
    dev_free(&t.chirp);
    dev_free(&t.bhat);
    dev_free(&t.cs);
    dev_free(&t.stages);
  }
  for (auto& s : pl->subs)
    for (auto& b : s.lam) dev_free(&b);
  for (auto& bp : pl->batch.passes) {
    dev_free(&bp.args);
    for (auto& g : bp.groups) {
      dev_free(&g.tile_prob);
      dev_free(&g.tile_idx);
    }
  }
  if (pl->batch.staging) (void)hipHostFree(pl->batch.staging);
  if (pl->batch.uploaded) (void)hipEventDestroy(pl->batch.uploaded);
  for (hipStream_t t : pl->batch.side) (void)hipStreamDestroy(t);
  if (pl->batch.fork) (void)hipEventDestroy(pl->batch.fork);
  for (hipEvent_t e : pl->batch.join) (void)hipEventDestroy(e);
  for (DevBuf* b : {&pl->batch.rhs_tab, &pl->batch.phi_tab, &pl->batch.work_tab, &pl->batch.resid_args,
                    &pl->batch.blk_prob, &pl->batch.blk_start, &pl->batch.blk_count, &pl->batch.inv_wsum,
                    &pl->batch.partials})
    dev_free(b);
  dev_free(&pl->work);
  dev_free(&pl->partials);
  dev_free(&pl->scalars);
  dev_free(&pl->proj_g);
  for (auto& r : pl->prof) (void)hipEventDestroy(r.end);
  if (pl->prof_start) (void)hipEventDestroy(pl->prof_start);
  if (pl->graph.exec) (void)hipGraphExecDestroy(pl->graph.exec);
  if (pl->graph.graph) (void)hipGraphDestroy(pl->graph.graph);
  if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
  tune_end(pl->tune);
  for (void* c : pl->pool) (void)hipFree(c);
  delete pl;
}

mpois_status build_batch(mpois_plan_s* pl);

mpois_status create_common(const mpois_grid_desc* gs, int count, int approx, int prec, double rtol, int max_iter,
                           unsigned flags, mpois_plan* out) {
  if (!out || !gs || count < 1 || count > 2048) return MPOIS_ERR_INVALID;
  if (!(std::isfinite(rtol) && rtol >= 0)) return MPOIS_ERR_INVALID;
  int64_t maxpts = 0;
  for (int i = 0; i < count; ++i) {
    mpois_status st = validate_one(&gs[i], approx, prec, max_iter);
    if (st != MPOIS_OK) return st;
    if (gs[i].ndim != gs[0].ndim) return MPOIS_ERR_INVALID;
  }
  int dev = 0;
  mpois_status st = device_ready(&dev);
  if (st != MPOIS_OK) return st;
  mpois_plan_s* pl = new (std::nothrow) mpois_plan_s();
  if (!pl) return MPOIS_ERR_NOMEM;
  pl->approx = approx;
  pl->prec = prec;
  pl->rtol = rtol;
  pl->max_iter = prec == MPOIS_F32_REFINE ? max_iter : 0;
  pl->flags = flags;
  pl->device = dev;
  pl->f64work = prec == MPOIS_F64 || (prec == MPOIS_F32_REFINE && (flags & MPOIS_FLAG_F64_ARITH));
  pl->subs.resize(size_t(count));
  for (int i = 0; i < count && st == MPOIS_OK; ++i) {
    st = build_sub(pl, &gs[i], &pl->subs[i]);
    maxpts = std::max(maxpts, pl->subs[i].npts);
  }
  tune_end(pl->tune);
  pl->tune = nullptr;
  int64_t total_pts = 0;
  for (auto& sp : pl->subs) total_pts += sp.npts;
  const int64_t work_pts = count > 1 ? total_pts : maxpts;
  if (st == MPOIS_OK && prec == MPOIS_F32_REFINE) st = dev_alloc(pl, &pl->work, size_t(work_pts) * sizeof(float));
  if (st == MPOIS_OK && count > 1) st = build_batch(pl);
  if (st == MPOIS_OK) st = dev_alloc(pl, &pl->partials, size_t(kMaxResidBlocks) * 4 * sizeof(double));
  if (st == MPOIS_OK) st = dev_alloc(pl, &pl->scalars, size_t(count) * S_COUNT * sizeof(double));
  if (st == MPOIS_OK && (flags & MPOIS_FLAG_GRAPH)) {
    if (hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking) != hipSuccess) st = MPOIS_ERR_DEVICE;
  }
  if (st != MPOIS_OK) {
    free_plan(pl);
    return st;
  }
  *out = pl;
  return MPOIS_OK;
}

// ---------------------------------------------------------------------------- execution
void prof_mark(mpois_plan_s* pl, int kernel, double bytes, hipStream_t s) {
  if (!pl->profiling) return;
  if (pl->prof_used == pl->prof.size()) {
    ProfRec r{};
    if (hipEventCreate(&r.end) != hipSuccess) return;
    pl->prof.push_back(r);
  }
  ProfRec& r = pl->prof[pl->prof_used++];
  r.kernel = kernel;
  r.bytes = bytes;
  (void)hipEventRecord(r.end, s);
}

// Element strides of the caller's arrays, padded to 3D (leading unit axes), or
// null for C-contiguous arrays.
struct IoViews {
  const int64_t* rhs = nullptr;
  const int64_t* phi = nullptr;
};

// Addressing of one array in a pass along padded axis `ax`: lines enumerate
// the other two axes (oa outer, ob inner).
void set_view(int ax, const int64_t n[3], const int64_t st[3], int64_t* vnb, int64_t* va, int64_t* vb, int64_t* vd) {
  const int oa = ax == 0 ? 1 : 0, ob = ax == 2 ? 1 : 2;
  *vnb = n[ob];
  *va = st[oa];
  *vb = st[ob];
  *vd = st[ax];
}

hipError_t run_solve(mpois_plan_s* pl, SubPlan& sp, const void* in, int in_f64, void* out, int out_f64, void* work,
                     int work_f64, bool update, const double* shift, hipStream_t s,
                     const int64_t* in_view = nullptr, const int64_t* out_view = nullptr,
                     const int64_t* work_view = nullptr, const ProjDev* proj = nullptr) {
  TraceRange trace_("mpois: solve");
  const size_t np = sp.passes.size();
  if (sp.plane >= 0 && !in_view && !out_view && !work_view && !proj) {
    // forward planes (axes 2 and 1), the fused axis-0 sweep, inverse planes
    const double pts = double(sp.npts);
    PassArgs f2 = sp.passes[0].args, f1 = sp.passes[1].args;
    f2.src = in;
    f2.src_f64 = in_f64;
    f1.dst = work;
    f1.dst_f64 = work_f64;
    hipError_t e = launch_plane(sp.plane, f2, f1, 0, sp.n[0], s);
    if (e != hipSuccess) return e;
    prof_mark(pl, kPlaneBase + sp.plane, pts * ((in_f64 ? 8 : 4) + (work_f64 ? 8 : 4)), s);
    Pass& m = sp.passes[2];
    PassArgs a = m.args;
    a.src = a.dst = work;
    a.src_f64 = a.dst_f64 = work_f64;
    e = m.spec >= 0 ? launch_spec(m.spec, a, s) : launch_line_pass(m.cfg, a, s);
    if (e != hipSuccess) return e;
    prof_mark(pl, m.spec >= 0 ? kSpecBase + m.spec : m.cfg, pts * (work_f64 ? 16 : 8), s);
    PassArgs i1 = sp.passes[3].args, i2 = sp.passes[4].args;
    i1.src = work;
    i1.src_f64 = work_f64;
    i2.dst = out;
    i2.dst_f64 = out_f64;
    i2.update = update ? 1 : 0;
    i2.shift = shift;
    e = launch_plane(sp.plane, i2, i1, 1, sp.n[0], s);
    if (e != hipSuccess) return e;
    prof_mark(pl, kPlaneBase + sp.plane, pts * ((work_f64 ? 8 : 4) + (out_f64 ? 8 : 4) + (update ? 8 : 0)), s);
    return hipSuccess;
  }
  for (size_t i = 0; i < np; ++i) {
    Pass& p = sp.passes[i];
    PassArgs a = p.args;
    a.src = i == 0 ? in : work;
    a.src_f64 = i == 0 ? in_f64 : work_f64;
    const bool last = i + 1 == np;
    a.dst = last ? out : work;
    a.dst_f64 = last ? out_f64 : work_f64;
    const int64_t* sv = i == 0 ? in_view : work_view;
    const int64_t* dv = last ? out_view : work_view;
    const int axp = 3 - sp.ndim + p.axis;
    if (sv) set_view(axp, sp.n, sv, &a.src_vnb, &a.src_va, &a.src_vb, &a.src_vd);
    if (dv) set_view(axp, sp.n, dv, &a.dst_vnb, &a.dst_va, &a.dst_vb, &a.dst_vd);
    a.contig = (sv || dv) ? 0 : 1;
    a.update = (last && update) ? 1 : 0;
    a.shift = shift;
    if (proj) {
      // projection step: the first pass forms div(vel) / adt as it loads, the
      // last one corrects p and the last-axis velocity component as it stores
      a.proj = *proj;
      a.proj_load = i == 0 ? 1 : 0;
      a.proj_store = last ? 1 : 0;
      if (a.proj_load || a.proj_store) a.contig = 0;
    }
    // the specialised kernels take the contiguous tile paths when they can, and
    // their generic path otherwise (views included)
    // (the projection loads and stores exist in the generic kernels and the
    // unfused specialised ones)
    const bool spec = p.spec >= 0 && !((a.proj_load || a.proj_store) && a.kind_b >= 0);
    hipError_t e = spec ? launch_spec(p.spec, a, s) : launch_line_pass(p.cfg, a, s);
    if (e != hipSuccess) return e;
    const double pts = double(sp.npts);
    prof_mark(pl, spec ? kSpecBase + p.spec : p.cfg, pts * ((a.src_f64 ? 8 : 4) + (a.dst_f64 ? 8 : 4) + (a.update ? 8 : 0)), s);
  }
  return hipSuccess;
}

// Scratch of one single-grid execute: the FP32 working array of refinement
// plans, the residual kernel's block partial sums (kMaxResidBlocks x 4) and
// the reduced scalars (S_COUNT per grid).
struct Workspace {
  void* work;
  double* partials;
  double* scalars;
};

Workspace plan_workspace(mpois_plan_s* pl) {
  return {pl->work.p, static_cast<double*>(pl->partials.p), static_cast<double*>(pl->scalars.p)};
}

hipError_t run_resid(mpois_plan_s* pl, SubPlan& sp, const void* rhs, const void* phi, void* r, int r_f64,
                     const double* mg, double* scalars, hipStream_t s, double* partials = nullptr,
                     const IoViews& views = IoViews()) {
  TraceRange trace_("mpois: residual");
  ResidArgs a = sp.resid;
  for (int e = 0; e < 3; ++e) {
    if (views.phi) a.ps[e] = views.phi[sp.rperm[e]];
    if (views.rhs) a.gs[e] = views.rhs[sp.rperm[e]];
  }
  a.phi = static_cast<const double*>(phi);
  a.g = static_cast<const double*>(rhs);
  a.r = r;
  a.r_f64 = r_f64;
  a.mg = mg;
  a.partials = partials ? partials : static_cast<double*>(pl->partials.p);
  hipError_t e = launch_resid(a, s);
  if (e != hipSuccess) return e;
  prof_mark(pl, 100, double(sp.npts) * (phi ? 16 : 8) + (r ? double(sp.npts) * (r_f64 ? 8 : 4) : 0), s);
  e = launch_finalize(a.partials, resid_blocks(a.n), 1.0 / sp.wsum, scalars, s);
  if (e != hipSuccess) return e;
  prof_mark(pl, 101, double(resid_blocks(a.n)) * 32, s);
  return hipSuccess;
}

hipError_t enqueue_one(mpois_plan_s* pl, SubPlan& sp, size_t sub_index, const void* rhs, void* phi, hipStream_t s,
                       const Workspace& ws, const IoViews& v = IoViews()) {
  // F64 / F32: every sweep works in place on phi (through its view)
  if (pl->prec == MPOIS_F64) return run_solve(pl, sp, rhs, 1, phi, 1, phi, 1, false, nullptr, s, v.rhs, v.phi, v.phi);
  if (pl->prec == MPOIS_F32) return run_solve(pl, sp, rhs, 0, phi, 0, phi, 0, false, nullptr, s, v.rhs, v.phi, v.phi);
  // FP32 solve, then fixed number of FP64-residual corrections.
  double* sc = ws.scalars + sub_index * S_COUNT;
  void* work = ws.work;
  hipError_t e;
  if (sp.singular) {
    // m_g = sum w g / sum w, so the FP32 residual carries no large constant.
    if ((e = run_resid(pl, sp, rhs, nullptr, nullptr, 0, nullptr, sc, s, ws.partials, v)) != hipSuccess) return e;
  }
  if ((e = run_solve(pl, sp, rhs, 1, phi, 1, work, 0, false, nullptr, s, v.rhs, v.phi, nullptr)) != hipSuccess)
    return e;
  for (int it = 0; it < pl->max_iter; ++it) {
    // r = g - m_g - L phi (FP64, stored FP32), sum w phi -> gauge shift
    if ((e = run_resid(pl, sp, rhs, phi, work, 0, sp.singular ? sc + S_MG : nullptr, sc, s, ws.partials, v)) !=
        hipSuccess)
      return e;
    // phi <- phi + delta, minus the weighted mean of phi when the problem is singular
    if ((e = run_solve(pl, sp, work, 0, phi, 1, work, 0, true, sp.singular ? sc + S_SHIFT : nullptr, s, nullptr, v.phi,
                       nullptr)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

mpois_status build_batch(mpois_plan_s* pl) {
  BatchState& B = pl->batch;
  pl->batched = true;
  const int count = int(pl->subs.size());
  const size_t npass = pl->subs[0].passes.size();
  B.passes.resize(npass);
  for (size_t p = 0; p < npass; ++p) {
    BatchPass& bp = B.passes[p];
    std::vector<PassArgs> args(static_cast<size_t>(count));
    std::map<int, std::pair<std::vector<int>, std::vector<int>>> by_cfg;  // cfg -> (tile_prob, tile_idx)
    std::map<int, size_t> lds_of;
    for (int i = 0; i < count; ++i) {
      const Pass& ps = pl->subs[i].passes[p];
      args[i] = ps.args;
      int cf64, np, nt, pmax;
      kernel_cfg(ps.cfg, &cf64, &np, &nt, &pmax);
      const int64_t tiles = (ps.args.nlines + 2 * np - 1) / (2 * np);
      auto& lists = by_cfg[ps.cfg];
      for (int64_t t = 0; t < tiles; ++t) {
        lists.first.push_back(i);
        lists.second.push_back(int(t));
      }
      lds_of[ps.cfg] = std::max(lds_of[ps.cfg], line_pass_lds(ps.cfg, ps.args.ax.n, ps.args.ax.P));
    }
    mpois_status st = dev_upload(pl, &bp.args, args);
    if (st != MPOIS_OK) return st;
    for (auto& kv : by_cfg) {
      BatchGroup g;
      g.cfg = kv.first;
      g.blocks = int(kv.second.first.size());
      g.lds = lds_of[kv.first];
      if ((st = dev_upload(pl, &g.tile_prob, kv.second.first)) != MPOIS_OK) return st;
      if ((st = dev_upload(pl, &g.tile_idx, kv.second.second)) != MPOIS_OK) return st;
      bp.groups.push_back(g);
    }
  }
  // residual blocks: about 8k points each, 1..256 per grid
  std::vector<ResidArgs> rargs(static_cast<size_t>(count));
  std::vector<int> blk_prob, blk_start(static_cast<size_t>(count)), blk_count(static_cast<size_t>(count));
  std::vector<double> inv_wsum(static_cast<size_t>(count));
  for (int i = 0; i < count; ++i) {
    const SubPlan& sp = pl->subs[i];
    rargs[i] = sp.resid;
    rargs[i].singular = sp.singular ? 1 : 0;
    B.any_singular = B.any_singular || sp.singular;
    const int64_t* rn = sp.resid.n;
    const int64_t units = rn[1] * ((rn[2] + 255) / 256) * ((rn[0] + 31) / 32);  // residual work units
    int64_t nb = (sp.npts + 8191) / 8192;
    nb = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(nb, 256), units));
    blk_start[i] = int(blk_prob.size());
    blk_count[i] = int(nb);
    for (int64_t b = 0; b < nb; ++b) blk_prob.push_back(i);
    inv_wsum[i] = 1.0 / sp.wsum;
  }
  B.resid_blocks = int(blk_prob.size());
  mpois_status st = dev_upload(pl, &B.resid_args, rargs);
  if (st == MPOIS_OK) st = dev_upload(pl, &B.blk_prob, blk_prob);
  if (st == MPOIS_OK) st = dev_upload(pl, &B.blk_start, blk_start);
  if (st == MPOIS_OK) st = dev_upload(pl, &B.blk_count, blk_count);
  if (st == MPOIS_OK) st = dev_upload(pl, &B.inv_wsum, inv_wsum);
  if (st == MPOIS_OK) st = dev_alloc(pl, &B.partials, size_t(B.resid_blocks) * 4 * sizeof(double));
  if (st == MPOIS_OK) st = dev_alloc(pl, &B.rhs_tab, size_t(count) * sizeof(void*));
  if (st == MPOIS_OK) st = dev_alloc(pl, &B.phi_tab, size_t(count) * sizeof(void*));
  if (st != MPOIS_OK) return st;
  if (fault_alloc() || hipHostMalloc(reinterpret_cast<void**>(&B.staging), 2 * size_t(count) * sizeof(void*),
                                     hipHostMallocDefault) != hipSuccess) {
    B.staging = nullptr;
    (void)hipGetLastError();
    return MPOIS_ERR_NOMEM;
  }
  if (hipEventCreateWithFlags(&B.uploaded, hipEventDisableTiming) != hipSuccess) return MPOIS_ERR_DEVICE;
  size_t max_groups = 0;
  for (const BatchPass& bp : B.passes) max_groups = std::max(max_groups, bp.groups.size());
  constexpr size_t kSide = 3;
  const size_t nside = std::min(kSide, max_groups > 0 ? max_groups - 1 : 0);
  if (nside > 0 && hipEventCreateWithFlags(&B.fork, hipEventDisableTiming) != hipSuccess) return MPOIS_ERR_DEVICE;
  for (size_t i = 0; i < nside; ++i) {
    hipStream_t t = nullptr;
    hipEvent_t e = nullptr;
    if (hipStreamCreateWithFlags(&t, hipStreamNonBlocking) != hipSuccess) return MPOIS_ERR_DEVICE;
    B.side.push_back(t);
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return MPOIS_ERR_DEVICE;
    B.join.push_back(e);
  }
  if (pl->prec == MPOIS_F32_REFINE) {
    std::vector<void*> work(static_cast<size_t>(count));
    int64_t off = 0;
    for (int i = 0; i < count; ++i) {
      work[i] = static_cast<float*>(pl->work.p) + off;
      off += pl->subs[i].npts;
    }
    if ((st = dev_upload(pl, &B.work_tab, work)) != MPOIS_OK) return st;
  }
  return MPOIS_OK;
}

// All passes of one solve over every grid of a batch.  src/dst tables per pass:
// first pass reads `in`, last pass writes `out`, the others use `work`.
hipError_t batch_solve(mpois_plan_s* pl, const void* const* in, int in_f64, void* const* out, int out_f64,
                       void* const* work, int work_f64, bool update, hipStream_t s) {
  TraceRange trace_("mpois: batch solve");
  BatchState& B = pl->batch;
  const size_t np = B.passes.size();
  for (size_t p = 0; p < np; ++p) {
    BatchPassArgs b{};
    b.args = static_cast<const PassArgs*>(B.passes[p].args.p);
    b.src_tab = p == 0 ? in : static_cast<const void* const*>(work);
    b.src_f64 = p == 0 ? in_f64 : work_f64;
    const bool last = p + 1 == np;
    b.dst_tab = last ? out : work;
    b.dst_f64 = last ? out_f64 : work_f64;
    b.update = (last && update) ? 1 : 0;
    b.shift_base = static_cast<const double*>(pl->scalars.p) + S_SHIFT;
    b.shift_stride = S_COUNT;
    const auto& groups = B.passes[p].groups;
    const size_t nside = std::min(B.side.size(), groups.size() > 0 ? groups.size() - 1 : 0);
    hipError_t e = hipSuccess;
    if (nside > 0) {
      if ((e = hipEventRecord(B.fork, s)) != hipSuccess) return e;
      for (size_t k = 0; k < nside; ++k)
        if ((e = hipStreamWaitEvent(B.side[k], B.fork, 0)) != hipSuccess) return e;
    }
    for (size_t i = 0; i < groups.size(); ++i) {
      const BatchGroup& g = groups[i];
      b.tile_prob = static_cast<const int*>(g.tile_prob.p);
      b.tile_idx = static_cast<const int*>(g.tile_idx.p);
      hipStream_t t = (i == 0 || nside == 0) ? s : B.side[(i - 1) % nside];
      if ((e = launch_line_pass_batch(g.cfg, b, g.blocks, g.lds, t)) != hipSuccess) return e;
    }
    for (size_t k = 0; k < nside; ++k) {
      if ((e = hipEventRecord(B.join[k], B.side[k])) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(s, B.join[k], 0)) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t batch_resid(mpois_plan_s* pl, const void* const* phi, const void* const* g, void* const* r, bool use_mg,
                       hipStream_t s) {
  TraceRange trace_("mpois: batch residual");
  BatchState& B = pl->batch;
  BatchResidArgs b{};
  b.args = static_cast<const ResidArgs*>(B.resid_args.p);
  b.blk_prob = static_cast<const int*>(B.blk_prob.p);
  b.blk_start = static_cast<const int*>(B.blk_start.p);
  b.blk_count = static_cast<const int*>(B.blk_count.p);
  b.phi_tab = phi;
  b.g_tab = g;
  b.r_tab = r;
  b.r_f64 = 0;
  b.use_mg = use_mg ? 1 : 0;
  b.scalars = static_cast<double*>(pl->scalars.p);
  b.partials = static_cast<double*>(B.partials.p);
  hipError_t e = launch_resid_batch(b, B.resid_blocks, s);
  if (e != hipSuccess) return e;
  return launch_finalize_batch(b.partials, b.blk_start, b.blk_count, static_cast<const double*>(B.inv_wsum.p),
                               b.scalars, int(pl->subs.size()), s);
}

// The kernels of one batched execute; they read the array pointers from the
// device tables, so the same sequence (or its captured graph) serves any
// pointers once the tables hold them.
hipError_t enqueue_batch(mpois_plan_s* pl, hipStream_t s) {
  BatchState& B = pl->batch;
  hipError_t e = hipSuccess;
  auto rhs = static_cast<const void* const*>(B.rhs_tab.p);
  auto phi = static_cast<void* const*>(B.phi_tab.p);
  if (pl->prec == MPOIS_F64) return batch_solve(pl, rhs, 1, phi, 1, phi, 1, false, s);
  if (pl->prec == MPOIS_F32) return batch_solve(pl, rhs, 0, phi, 0, phi, 0, false, s);
  auto work = static_cast<void* const*>(B.work_tab.p);
  if (B.any_singular && (e = batch_resid(pl, nullptr, rhs, nullptr, false, s)) != hipSuccess) return e;
  if ((e = batch_solve(pl, rhs, 1, phi, 1, work, 0, false, s)) != hipSuccess) return e;
  for (int it = 0; it < pl->max_iter; ++it) {
    if ((e = batch_resid(pl, static_cast<const void* const*>(static_cast<const void*>(phi)), rhs, work, true, s)) !=
        hipSuccess)
      return e;
    if ((e = batch_solve(pl, static_cast<const void* const*>(static_cast<const void*>(work)), 0, phi, 1, work, 0,
                         true, s)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

}  // namespace

// The gauge pass above runs the residual kernel without phi: it only forms
// sum w g (S_WG, S_MG) and sum g^2.

extern "C" {

const char* mpois_status_string(mpois_status s) {
  // a C caller may pass any int: read the bits, not a (possibly out of
  // range) enumerator
  int v;
  std::memcpy(&v, &s, sizeof v);
  switch (v) {
    case MPOIS_OK: return "ok";
    case MPOIS_ERR_INVALID: return "invalid argument";
    case MPOIS_ERR_UNSUPPORTED: return "unsupported";
    case MPOIS_ERR_NOMEM: return "out of device memory";
    case MPOIS_ERR_DEVICE: return "device error";
    case MPOIS_ERR_NOT_CONVERGED: return "refinement did not reach rtol";
    case MPOIS_ERR_NONFINITE: return "non-finite residual";
  }
  return "unknown status";
}

mpois_status mpois_validate(const mpois_grid_desc* grid, int approx, int prec, int max_iter) {
  return validate_one(grid, approx, prec, max_iter);
}

mpois_status mpois_axis_eigenvalues(int bc, int grid, int approx, int64_t n, double h, double* out) {
  if (!out || n < 1 || bc < 0 || bc > MPOIS_AXIS_ND || (grid != 0 && grid != 1) || !(h > 0 && std::isfinite(h)))
    return MPOIS_ERR_INVALID;
  if (approx != MPOIS_SPECTRAL && approx != MPOIS_FD2) return MPOIS_ERR_INVALID;
  if (bc == MPOIS_NEUMANN && grid == MPOIS_VERTEX && n < 2) return MPOIS_ERR_INVALID;
  axis_eigs(bc, bc == MPOIS_PERIODIC ? MPOIS_VERTEX : grid, approx, n, h, out);
  return MPOIS_OK;
}

mpois_status mpois_axis_plan(int bc, int grid, int64_t n, int* kind_fwd, int* kind_bwd, int* M, int* P, int* radices,
                             int cap, int* nradix) {
  if (n < 1 || bc < 0 || bc > MPOIS_AXIS_ND || (grid != 0 && grid != 1)) return MPOIS_ERR_INVALID;
  if (bc == MPOIS_NEUMANN && grid == MPOIS_VERTEX && n < 2) return MPOIS_ERR_INVALID;
  AxisShape s = plan_axis_shape(bc, bc == MPOIS_PERIODIC ? MPOIS_VERTEX : grid, n, true);
  if (kind_fwd) *kind_fwd = s.kind_f;
  if (kind_bwd) *kind_bwd = s.kind_b;
  if (M) *M = int(s.M);
  if (P) *P = int(s.P);
  if (nradix) *nradix = int(s.radices.size());
  if (radices)
    for (int i = 0; i < cap && i < int(s.radices.size()); ++i) radices[i] = s.radices[i];
  return MPOIS_OK;
}

mpois_status mpois_plan_create(const mpois_grid_desc* grid, int approx, int prec, double rtol, int max_iter,
                               unsigned flags, mpois_plan* out) {
  TraceRange trace_("mpois_plan_create");
  return create_common(grid, 1, approx, prec, rtol, max_iter, flags, out);
}

mpois_status mpois_plan_create_batch(const mpois_grid_desc* grids, int count, int approx, int prec, double rtol,
                                     int max_iter, unsigned flags, mpois_plan* out) {
  TraceRange trace_("mpois_plan_create_batch");
  return create_common(grids, count, approx, prec, rtol, max_iter, flags, out);
}

static mpois_status check_ptrs(const mpois_plan_s* pl, const SubPlan& sp, const void* rhs, void* phi) {
  if (!rhs || !phi) return MPOIS_ERR_INVALID;
  const size_t es = pl->prec == MPOIS_F32 ? 4 : 8;
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(rhs), b0 = reinterpret_cast<uintptr_t>(phi);
  const uintptr_t len = uintptr_t(sp.npts) * es;
  if (a0 != b0 && a0 < b0 + len && b0 < a0 + len) return MPOIS_ERR_INVALID;
  if (a0 == b0 && pl->prec == MPOIS_F32_REFINE) return MPOIS_ERR_INVALID;
  for (const void* p : {rhs, static_cast<const void*>(phi)}) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
      (void)hipGetLastError();
      return MPOIS_ERR_INVALID;
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) return MPOIS_ERR_INVALID;
  }
  return MPOIS_OK;
}

mpois_status mpois_execute(mpois_plan pl, const void* rhs, void* phi, void* stream) {
  TraceRange trace_("mpois_execute");
  if (!pl || pl->subs.size() != 1) return MPOIS_ERR_INVALID;
  SubPlan& sp = pl->subs[0];
  // the attribute queries are host calls: repeat them only for new pointers
  if (!(rhs && phi && rhs == pl->checked_rhs && phi == pl->checked_phi)) {
    mpois_status st = check_ptrs(pl, sp, rhs, phi);
    if (st != MPOIS_OK) return st;
    pl->checked_rhs = rhs;
    pl->checked_phi = phi;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  pl->last_rhs = rhs;
  pl->last_phi = phi;
  pl->last_view = false;
  pl->last_rhs_b.clear();
  pl->last_phi_b.clear();
  pl->last_iters = pl->prec == MPOIS_F32_REFINE ? 1 + pl->max_iter : 1;
  if (pl->flags & MPOIS_FLAG_PROFILE) {
    if (!pl->prof_start && hipEventCreate(&pl->prof_start) != hipSuccess) return MPOIS_ERR_DEVICE;
    pl->prof_used = 0;
    pl->profiling = true;
    (void)hipEventRecord(pl->prof_start, s);
    const hipError_t e = enqueue_one(pl, sp, 0, rhs, phi, s, plan_workspace(pl));
    pl->profiling = false;
    return e == hipSuccess ? MPOIS_OK : MPOIS_ERR_DEVICE;
  }
  if (pl->flags & MPOIS_FLAG_GRAPH) {
    Graph& g = pl->graph;
    if (!(g.exec && g.rhs == rhs && g.phi == phi)) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      if (g.graph) (void)hipGraphDestroy(g.graph);
      g.exec = nullptr;
      g.graph = nullptr;
      if (hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return MPOIS_ERR_DEVICE;
      hipError_t e = enqueue_one(pl, sp, 0, rhs, phi, pl->cap_stream, plan_workspace(pl));
      hipGraph_t graph = nullptr;
      hipError_t e2 = hipStreamEndCapture(pl->cap_stream, &graph);
      if (e != hipSuccess || e2 != hipSuccess || !graph) return MPOIS_ERR_DEVICE;
      g.graph = graph;
      if (hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess) return MPOIS_ERR_DEVICE;
      g.rhs = rhs;
      g.phi = phi;
    }
    return hipGraphLaunch(g.exec, s) == hipSuccess ? MPOIS_OK : MPOIS_ERR_DEVICE;
  }
  return enqueue_one(pl, sp, 0, rhs, phi, s, plan_workspace(pl)) == hipSuccess ? MPOIS_OK : MPOIS_ERR_DEVICE;
}

// Batched plans: the pointer arrays are validated and uploaded only when they
// differ from the previous call's (pinned staging, asynchronous copy on the
// execute's stream); with MPOIS_FLAG_GRAPH the kernel sequence is captured
// once and replayed, since it reads the pointers from the device tables.
static mpois_status batch_set_tables(mpois_plan_s* pl, const void* const* rhs, void* const* phi, hipStream_t s) {
  BatchState& B = pl->batch;
  const size_t count = pl->subs.size();
  if (B.have_tables && std::equal(rhs, rhs + count, B.staging) && std::equal(phi, phi + count, B.staging + count))
    return MPOIS_OK;
  for (size_t i = 0; i < count; ++i) {
    mpois_status st = check_ptrs(pl, pl->subs[i], rhs[i], phi[i]);
    if (st != MPOIS_OK) return st;
  }
  // the previous upload must have left the staging buffer before it is rewritten
  if (B.have_tables && hipEventSynchronize(B.uploaded) != hipSuccess) return MPOIS_ERR_DEVICE;
  B.have_tables = false;
  for (size_t i = 0; i < count; ++i) {
    B.staging[i] = const_cast<void*>(rhs[i]);
    B.staging[count + i] = phi[i];
  }
  const size_t tb = count * sizeof(void*);
  if (hipMemcpyAsync(B.rhs_tab.p, B.staging, tb, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(B.phi_tab.p, B.staging + count, tb, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipEventRecord(B.uploaded, s) != hipSuccess)
    return MPOIS_ERR_DEVICE;
  B.have_tables = true;
  return MPOIS_OK;
}

// ---------------------------------------------------------------------------- views into larger arrays
// Checks of one view: strides of a row-major-like, non-self-overlapping layout
// (s[d] >= s[d+1] n[d+1] >= 1); padded to 3D; extent in elements.
static mpois_status view_strides(const SubPlan& sp, const int64_t* st, int64_t out[3], int64_t* extent) {
  const int D = sp.ndim;
  for (int d = 0; d < D; ++d)
    if (st[d] < 1) return MPOIS_ERR_INVALID;
  for (int d = 0; d + 1 < D; ++d)
    if (st[d] < st[d + 1] * sp.n[3 - D + d + 1]) return MPOIS_ERR_INVALID;
  int64_t ext = 1;
  for (int e = 0; e < 3; ++e) {
    const int d = e - (3 - D);
    out[e] = d >= 0 ? st[d] : st[0] * sp.n[3 - D];
    if (d >= 0) ext += (sp.n[e] - 1) * st[d];
  }
  *extent = ext;
  return MPOIS_OK;
}

mpois_status mpois_execute_view(mpois_plan pl, const void* rhs, const int64_t* rhs_strides, void* phi,
                                const int64_t* phi_strides, void* stream) {
  TraceRange trace_("mpois_execute_view");
  if (!pl || pl->subs.size() != 1 || !rhs || !phi || !rhs_strides || !phi_strides) return MPOIS_ERR_INVALID;
  SubPlan& sp = pl->subs[0];
  int64_t rs[3], ps[3], rext = 0, pext = 0;
  mpois_status st = view_strides(sp, rhs_strides, rs, &rext);
  if (st == MPOIS_OK) st = view_strides(sp, phi_strides, ps, &pext);
  if (st != MPOIS_OK) return st;
  const size_t es = pl->prec == MPOIS_F32 ? 4 : 8;
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(rhs), b0 = reinterpret_cast<uintptr_t>(phi);
  const bool same = a0 == b0 && std::equal(rs, rs + 3, ps);
  if (same && pl->prec == MPOIS_F32_REFINE) return MPOIS_ERR_INVALID;
  if (!same && a0 < b0 + uintptr_t(pext) * es && b0 < a0 + uintptr_t(rext) * es) return MPOIS_ERR_INVALID;
  for (const void* p : {rhs, static_cast<const void*>(phi)}) {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
      (void)hipGetLastError();
      return MPOIS_ERR_INVALID;
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) return MPOIS_ERR_INVALID;
  }
  pl->last_rhs = rhs;
  pl->last_phi = phi;
  pl->last_rhs_b.clear();
  pl->last_phi_b.clear();
  std::copy(rs, rs + 3, pl->last_rhs_view);
  std::copy(ps, ps + 3, pl->last_phi_view);
  pl->last_view = true;
  pl->last_iters = pl->prec == MPOIS_F32_REFINE ? 1 + pl->max_iter : 1;
  IoViews v;
  v.rhs = pl->last_rhs_view;
  v.phi = pl->last_phi_view;
  return enqueue_one(pl, sp, 0, rhs, phi, static_cast<hipStream_t>(stream), plan_workspace(pl), v) == hipSuccess
             ? MPOIS_OK
             : MPOIS_ERR_DEVICE;
}

// Projection step of an incompressible-flow solver on the plan's staggered
// grid (paper Section 5.1): Lap phi = div(u*) / adt, u = u* - adt grad phi,
// p += phi.  FP64 / FP32 plans fuse the divergence into the first line pass
// and the pressure update and the last-axis velocity correction into the
// last; the other velocity components take one more kernel.  Refinement
// plans need the right-hand side as an FP64 array for their residuals: the
// divergence is formed into a plan buffer (allocated on the first call),
// solved with refinement, and all of the correction runs afterwards.
mpois_status mpois_project(mpois_plan pl, void* const* vel, void* p, double adt, void* phi, void* stream) {
  TraceRange trace_("mpois_project");
  if (!pl || pl->subs.size() != 1 || pl->batched) return MPOIS_ERR_INVALID;
  SubPlan& sp = pl->subs[0];
  if (!vel || !p || !phi || !std::isfinite(adt) || !(adt > 0.0)) return MPOIS_ERR_INVALID;
  if (pl->approx != MPOIS_FD2 || sp.resid.shift != 0.0) return MPOIS_ERR_UNSUPPORTED;
  const int D = sp.ndim;
  const size_t es = pl->prec == MPOIS_F32 ? 4 : 8;
  ProjDev q{};
  for (int e = 0; e < 3; ++e) {
    q.n[e] = sp.n[e];
    q.inv_h[e] = 1.0 / sp.h[e];
  }
  std::vector<std::pair<uintptr_t, uintptr_t>> arrays;  // (address, bytes)
  int mask = 0;
  for (int d = 0; d < D; ++d) {
    const int e = 3 - D + d;
    const bool per = sp.face[e][0] == MPOIS_PERIODIC;
    if (!per && sp.grid[e] != MPOIS_STAGGERED) return MPOIS_ERR_UNSUPPORTED;
    if (!vel[d]) return MPOIS_ERR_INVALID;
    q.vel[e] = vel[d];
    q.ext[e] = per ? 0 : 1;
    q.dlo[e] = sp.face[e][0] == MPOIS_DIRICHLET ? 1 : 0;
    q.dhi[e] = sp.face[e][1] == MPOIS_DIRICHLET ? 1 : 0;
    int64_t shp[3] = {sp.n[0], sp.n[1], sp.n[2]};
    shp[e] += q.ext[e];
    q.vs[e][2] = 1;
    q.vs[e][1] = shp[2];
    q.vs[e][0] = shp[1] * shp[2];
    arrays.push_back({reinterpret_cast<uintptr_t>(vel[d]), uintptr_t(shp[0] * shp[1] * shp[2]) * es});
    mask |= 1 << e;
  }
  q.p = p;
  q.adt = adt;
  q.inv_adt = 1.0 / adt;
  arrays.push_back({reinterpret_cast<uintptr_t>(p), uintptr_t(sp.npts) * es});
  arrays.push_back({reinterpret_cast<uintptr_t>(phi), uintptr_t(sp.npts) * es});
  for (size_t i = 0; i < arrays.size(); ++i) {
    for (size_t j = i + 1; j < arrays.size(); ++j)
      if (arrays[i].first < arrays[j].first + arrays[j].second && arrays[j].first < arrays[i].first + arrays[i].second)
        return MPOIS_ERR_INVALID;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, reinterpret_cast<void*>(arrays[i].first)) != hipSuccess) {
      (void)hipGetLastError();
      return MPOIS_ERR_INVALID;
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged) return MPOIS_ERR_INVALID;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  pl->last_view = false;
  pl->last_rhs_b.clear();
  pl->last_phi_b.clear();
  if (pl->prec == MPOIS_F32_REFINE) {
    if (!pl->proj_g.p) {
      const mpois_status st = dev_alloc(pl, &pl->proj_g, size_t(sp.npts) * sizeof(double));
      if (st != MPOIS_OK) return st;
    }
    double* g = static_cast<double*>(pl->proj_g.p);
    if (launch_proj_div(q, g, s) != hipSuccess) return MPOIS_ERR_DEVICE;
    if (enqueue_one(pl, sp, 0, g, phi, s, plan_workspace(pl)) != hipSuccess) return MPOIS_ERR_DEVICE;
    if (launch_proj_correct(q, phi, 1, mask, 1, s) != hipSuccess) return MPOIS_ERR_DEVICE;
    pl->last_rhs = g;  // mpois_get_info reports on this solve
    pl->last_phi = phi;
    pl->last_iters = 1 + pl->max_iter;
    return MPOIS_OK;
  }
  const int f64 = pl->prec == MPOIS_F64 ? 1 : 0;
  if (run_solve(pl, sp, nullptr, f64, phi, f64, phi, f64, false, nullptr, s, nullptr, nullptr, nullptr, &q) !=
      hipSuccess)
    return MPOIS_ERR_DEVICE;
  mask &= ~4;  // the last pass corrected the last axis's component
  if (mask && launch_proj_correct(q, phi, f64, mask, 0, s) != hipSuccess) return MPOIS_ERR_DEVICE;
  pl->last_rhs = nullptr;  // the divergence was never stored
  pl->last_phi = phi;
  pl->last_iters = 1;
  return MPOIS_OK;
}


// ---------------------------------------------------------------------------- allocation-free execute
// Static scratch of mpois_execute_noalloc: every device the library runs on
// holds one copy until the process ends.  Layout: reduced scalars (256 B),
// residual block partial sums (kMaxResidBlocks x 4 doubles), then the FP32
// working array of a refinement plan.  Host code must not pass `scratch`
// itself to a kernel (its host-side name is not a device address): the
// per-device address comes from hipGetSymbolAddress.
constexpr size_t kNoallocScalars = 256;
constexpr size_t kNoallocPartials = size_t(kMaxResidBlocks) * 4 * sizeof(double);
static __device__ __align__(256) unsigned char scratch[MPOIS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, looked up once per device with
// that device current (the caller's current device).
static mpois_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return MPOIS_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return MPOIS_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MPOIS_OK;
}

mpois_status mpois_execute_noalloc(mpois_plan pl, const void* rhs, void* phi, void* stream) {
  TraceRange trace_("mpois_execute_noalloc");
  if (!pl || pl->subs.size() != 1) return MPOIS_ERR_INVALID;
  SubPlan& sp = pl->subs[0];
  const size_t work_bytes = pl->prec == MPOIS_F32_REFINE ? size_t(sp.npts) * sizeof(float) : 0;
  if (kNoallocScalars + kNoallocPartials + work_bytes > size_t(MPOIS_NOALLOC_SCRATCH_BYTES))
    return MPOIS_ERR_UNSUPPORTED;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != pl->device) return MPOIS_ERR_DEVICE;
  if (!(rhs && phi && rhs == pl->checked_rhs && phi == pl->checked_phi)) {
    mpois_status st = check_ptrs(pl, sp, rhs, phi);
    if (st != MPOIS_OK) return st;
    pl->checked_rhs = rhs;
    pl->checked_phi = phi;
  }
  void* base = nullptr;
  mpois_status st = scratch_address(dev, &base);
  if (st != MPOIS_OK) return st;
  // nothing in the scratch has to start at zero: the residual kernel writes
  // every partial the reduction reads, the reduction writes every scalar it
  // later reads, and the first sweep writes the working array before use
  char* b = static_cast<char*>(base);
  Workspace ws{b + kNoallocScalars + kNoallocPartials, reinterpret_cast<double*>(b + kNoallocScalars),
               reinterpret_cast<double*>(b)};
  pl->last_rhs = rhs;
  pl->last_phi = phi;
  pl->last_view = false;
  pl->last_rhs_b.clear();
  pl->last_phi_b.clear();
  pl->last_iters = pl->prec == MPOIS_F32_REFINE ? 1 + pl->max_iter : 1;
  return enqueue_one(pl, sp, 0, rhs, phi, static_cast<hipStream_t>(stream), ws) == hipSuccess ? MPOIS_OK
                                                                                              : MPOIS_ERR_DEVICE;
}

mpois_status mpois_execute_batch(mpois_plan pl, const void* const* rhs, void* const* phi, void* stream) {
  TraceRange trace_("mpois_execute_batch");
  if (!pl || !rhs || !phi) return MPOIS_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t count = pl->subs.size();
  if (!pl->batched) {
    mpois_status st = check_ptrs(pl, pl->subs[0], rhs[0], phi[0]);
    if (st != MPOIS_OK) return st;
  } else {
    mpois_status st = batch_set_tables(pl, rhs, phi, s);
    if (st != MPOIS_OK) return st;
  }
  pl->last_rhs = nullptr;
  pl->last_phi = nullptr;
  pl->last_view = false;
  pl->last_rhs_b.assign(rhs, rhs + count);
  pl->last_phi_b.assign(phi, phi + count);
  pl->last_iters = pl->prec == MPOIS_F32_REFINE ? 1 + pl->max_iter : 1;
  if (!pl->batched) return enqueue_one(pl, pl->subs[0], 0, rhs[0], phi[0], s, plan_workspace(pl)) == hipSuccess ? MPOIS_OK : MPOIS_ERR_DEVICE;
  if (pl->flags & MPOIS_FLAG_GRAPH) {
    Graph& g = pl->graph;
    if (!g.exec) {
      if (hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return MPOIS_ERR_DEVICE;
      hipError_t e = enqueue_batch(pl, pl->cap_stream);
      hipGraph_t graph = nullptr;
      hipError_t e2 = hipStreamEndCapture(pl->cap_stream, &graph);
      if (e != hipSuccess || e2 != hipSuccess || !graph) return MPOIS_ERR_DEVICE;
      g.graph = graph;
      if (hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess) return MPOIS_ERR_DEVICE;
    }
    return hipGraphLaunch(g.exec, s) == hipSuccess ? MPOIS_OK : MPOIS_ERR_DEVICE;
  }
  return enqueue_batch(pl, s) == hipSuccess ? MPOIS_OK : MPOIS_ERR_DEVICE;
}

mpois_status mpois_get_info(mpois_plan pl, void* stream, mpois_info* out) {
  TraceRange trace_("mpois_get_info");
  if (!pl || !out) return MPOIS_ERR_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  mpois_info info{};
  info.iters = pl->last_iters;
  info.rel_resid = std::nan("");
  info.zero_mode_rhs = 0.0;
  const bool batch = !pl->last_rhs_b.empty();
  const size_t count = batch ? pl->subs.size() : 1;
  if (!batch && !pl->last_rhs) return MPOIS_ERR_INVALID;
  if (pl->approx == MPOIS_FD2 && pl->prec != MPOIS_F32) {
    double worst = 0.0;
    double mg_worst = 0.0;
    for (size_t i = 0; i < count; ++i) {
      SubPlan& sp = pl->subs[i];
      const void* rhs = batch ? pl->last_rhs_b[i] : pl->last_rhs;
      const void* phi = batch ? pl->last_phi_b[i] : pl->last_phi;
      double* sc = static_cast<double*>(pl->scalars.p) + i * S_COUNT;
      IoViews v;
      if (!batch && pl->last_view) {
        v.rhs = pl->last_rhs_view;
        v.phi = pl->last_phi_view;
      }
      if (sp.singular && run_resid(pl, sp, rhs, nullptr, nullptr, 0, nullptr, sc, s, nullptr, v) != hipSuccess)
        return MPOIS_ERR_DEVICE;
      if (run_resid(pl, sp, rhs, phi, nullptr, 0, sp.singular ? sc + S_MG : nullptr, sc, s, nullptr, v) != hipSuccess)
        return MPOIS_ERR_DEVICE;
      double host[S_COUNT];
      if (hipMemcpyAsync(host, sc, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess) return MPOIS_ERR_DEVICE;
      if (hipStreamSynchronize(s) != hipSuccess) return MPOIS_ERR_DEVICE;
      const double rel = std::sqrt(host[S_R2]) / std::max(std::sqrt(host[S_G2]), 1e-300);
      const double mg = host[S_MG];
      if (i == 0 || !(rel <= worst)) {
        worst = rel;
        mg_worst = sp.singular ? mg : 0.0;
      }
    }
    info.rel_resid = worst;
    info.zero_mode_rhs = mg_worst;
  } else if (hipStreamSynchronize(s) != hipSuccess) {
    return MPOIS_ERR_DEVICE;
  }
  *out = info;
  if (!std::isfinite(info.rel_resid) && pl->approx == MPOIS_FD2 && pl->prec != MPOIS_F32) return MPOIS_ERR_NONFINITE;
  if (pl->rtol > 0 && pl->approx == MPOIS_FD2 && info.rel_resid > pl->rtol) return MPOIS_ERR_NOT_CONVERGED;
  return MPOIS_OK;
}

mpois_status mpois_destroy(mpois_plan pl) {
  if (!pl) return MPOIS_OK;
  free_plan(pl);
  return MPOIS_OK;
}

size_t mpois_workspace_bytes(mpois_plan pl) { return pl ? pl->bytes : 0; }

mpois_status mpois_kernel_shape(int cfg, int* elem_bytes, int* pairs, int* threads, int* max_len) {
  if (cfg >= kPlaneBase && cfg < kPlaneBase + num_planes()) {
    int f64, nt, n;
    plane_shape(cfg - kPlaneBase, &f64, &nt, &n);
    if (elem_bytes) *elem_bytes = f64 ? 8 : 4;
    if (pairs) *pairs = n / 2;
    if (threads) *threads = nt;
    if (max_len) *max_len = n;
    return MPOIS_OK;
  }
  if (cfg >= kSpecBase && cfg < kSpecBase + num_specs()) {
    int f64, np, nt, n;
    spec_shape(cfg - kSpecBase, &f64, &np, &nt, &n);
    if (elem_bytes) *elem_bytes = f64 ? 8 : 4;
    if (pairs) *pairs = np;
    if (threads) *threads = nt;
    if (max_len) *max_len = n;
    return MPOIS_OK;
  }
  if (cfg < 0 || cfg >= num_kernel_cfgs()) return MPOIS_ERR_INVALID;
  int f64, np, nt, pmax;
  kernel_cfg(cfg, &f64, &np, &nt, &pmax);
  if (elem_bytes) *elem_bytes = f64 ? 8 : 4;
  if (pairs) *pairs = np;
  if (threads) *threads = nt;
  if (max_len) *max_len = pmax;
  return MPOIS_OK;
}

mpois_status mpois_profile(mpois_plan pl, void* stream, int cap, double* ms, double* bytes, int* kernel, int* count) {
  if (!pl || !count || cap < 0) return MPOIS_ERR_INVALID;
  if (!(pl->flags & MPOIS_FLAG_PROFILE)) return MPOIS_ERR_INVALID;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return MPOIS_ERR_DEVICE;
  hipEvent_t prev = pl->prof_start;
  const int n = int(pl->prof_used);
  for (int i = 0; i < n && i < cap; ++i) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, prev, pl->prof[i].end) != hipSuccess) return MPOIS_ERR_DEVICE;
    if (ms) ms[i] = double(t);
    if (bytes) bytes[i] = pl->prof[i].bytes;
    if (kernel) kernel[i] = pl->prof[i].kernel;
    prev = pl->prof[i].end;
  }
  *count = n;
  return MPOIS_OK;
}

}  // extern "C"
