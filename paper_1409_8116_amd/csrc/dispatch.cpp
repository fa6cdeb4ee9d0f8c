// Kernel-shape table and dispatch of the line-transform kernel.
#include <hip/hip_runtime.h>

#include <vector>

#include "cfgs.h"
#include "internal.h"
#include "planes.h"
#include "specs.h"

namespace mpois {

// one set per shape, defined in lp_inst.hip compiled with MPOIS_CFG = shape id
#define MPOIS_DECL(I)                                                                                      \
  hipError_t launch_line_pass_cfg##I(const PassArgs& a, hipStream_t s, size_t lds);                        \
  hipError_t launch_line_pass_batch_cfg##I(const BatchPassArgs& b, int blocks, hipStream_t s, size_t lds); \
  hipError_t prepare_line_pass_cfg##I();
MPOIS_DECL(0) MPOIS_DECL(1) MPOIS_DECL(2) MPOIS_DECL(3) MPOIS_DECL(4) MPOIS_DECL(5) MPOIS_DECL(6)
MPOIS_DECL(7) MPOIS_DECL(8) MPOIS_DECL(9) MPOIS_DECL(10) MPOIS_DECL(11) MPOIS_DECL(12) MPOIS_DECL(13)
MPOIS_DECL(14) MPOIS_DECL(15) MPOIS_DECL(16) MPOIS_DECL(17)
#undef MPOIS_DECL

// one pair per specialised kernel, defined in sp_inst.hip compiled with MPOIS_SPEC = id
#define MPOIS_DECL_SPEC(ID, ...)                                                    \
  hipError_t launch_spec_##ID(const PassArgs& a, hipStream_t s, size_t lds); \
  hipError_t prepare_spec_##ID();
MPOIS_SPECS(MPOIS_DECL_SPEC)
#undef MPOIS_DECL_SPEC

// one per plane kernel, defined in pl_inst.hip
#define MPOIS_DECL_PLANE(ID, ...) \
  hipError_t launch_plane_##ID(const PassArgs& a2, const PassArgs& a1, int inverse, int64_t planes, hipStream_t s);
MPOIS_PLANES(MPOIS_DECL_PLANE)
#undef MPOIS_DECL_PLANE

namespace {
struct PlaneInfo {
  int f64, nt, n, M, P, kf, kb;
  std::vector<int> radices;
  hipError_t (*launch)(const PassArgs&, const PassArgs&, int, int64_t, hipStream_t);
};
const PlaneInfo kPlanes[] = {
#define X(ID, T, NT, N, M, P, KF, KB, ...) {sizeof(T) == 8, NT, N, M, P, KF, KB, {__VA_ARGS__}, &launch_plane_##ID},
    MPOIS_PLANES(X)
#undef X
};
constexpr int kNumPlanes = sizeof(kPlanes) / sizeof(kPlanes[0]);
static_assert(kNumPlanes == MPOIS_NUM_PLANES, "plane list and count disagree");

struct SpecInfo {
  int f64, np, nt, rader, pad, n, M, P, kf, kb;
  std::vector<int> radices;
  hipError_t (*launch)(const PassArgs&, hipStream_t, size_t);
  hipError_t (*prepare)();
};
const SpecInfo kSpecs[] = {
#define X(ID, T, NP, NT, RADER, SLIM, PAD, N, M, P, KF, KB, ...) \
  {sizeof(T) == 8, NP, NT, RADER, PAD, N, M, P, KF, KB, {__VA_ARGS__}, &launch_spec_##ID, &prepare_spec_##ID},
    MPOIS_SPECS(X)
#undef X
};
constexpr int kNumSpecs = sizeof(kSpecs) / sizeof(kSpecs[0]);
static_assert(kNumSpecs == MPOIS_NUM_SPECS, "spec list and count disagree");

struct KernelCfg {
  int f64, np, nt, pmax, rader, slim;
};
const KernelCfg kCfgs[] = {
#define X(ID, T, NP, NT, PMAX, RADER, SLIM) {sizeof(T) == 8, NP, NT, PMAX, RADER, SLIM},
    MPOIS_CFGS(X)
#undef X
};
constexpr int kNum = sizeof(kCfgs) / sizeof(kCfgs[0]);
static_assert(kNum == MPOIS_NUM_CFGS, "shape list and count disagree");
static_assert(kNum == 18, "update the per-shape function tables below");

using LaunchFn = hipError_t (*)(const PassArgs&, hipStream_t, size_t);
using LaunchBatchFn = hipError_t (*)(const BatchPassArgs&, int, hipStream_t, size_t);
using PrepareFn = hipError_t (*)();
#define MPOIS_ROW(F) \
  F##0, F##1, F##2, F##3, F##4, F##5, F##6, F##7, F##8, F##9, F##10, F##11, F##12, F##13, F##14, F##15, F##16, F##17
const LaunchFn kLaunch[kNum] = {MPOIS_ROW(launch_line_pass_cfg)};
const LaunchBatchFn kLaunchBatch[kNum] = {MPOIS_ROW(launch_line_pass_batch_cfg)};
const PrepareFn kPrepare[kNum] = {MPOIS_ROW(prepare_line_pass_cfg)};
#undef MPOIS_ROW
}  // namespace

int num_kernel_cfgs() { return kNum; }

void kernel_cfg(int i, int* f64, int* np, int* nt, int* pmax) {
  *f64 = kCfgs[i].f64;
  *np = kCfgs[i].np;
  *nt = kCfgs[i].nt;
  *pmax = kCfgs[i].pmax;
}

int kernel_cfg_rader(int i) { return kCfgs[i].rader; }
int kernel_cfg_slim(int i) { return kCfgs[i].slim; }

// LDS bytes: the larger of the real tile (2 NP rows, odd pitch) and the
// complex work buffer (NP pairs of P values).
size_t line_pass_lds(int cfg, int n, int P) {
  const KernelCfg& c = kCfgs[cfg];
  const size_t es = c.f64 ? 8 : 4;
  const size_t tl = 2 * size_t(c.np);
  const size_t xs = tl * size_t(n);
  const size_t zs = 2 * size_t(c.np) * size_t(P);
  return (xs > zs ? xs : zs) * es;
}

hipError_t prepare_kernels() {
  for (int i = 0; i < kNum; ++i) {
    hipError_t e = kPrepare[i]();
    if (e != hipSuccess) return e;
  }
  for (int i = 0; i < kNumSpecs; ++i) {
    hipError_t e = kSpecs[i].prepare();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int num_specs() { return kNumSpecs; }

// Specialised kernel for a pass with these parameters, or -1.
int find_spec(bool f64, int n, int M, int P, int kind_f, int kind_b, const std::vector<int>& radices) {
  for (int i = 0; i < kNumSpecs; ++i) {
    const SpecInfo& c = kSpecs[i];
    if ((c.f64 != 0) == f64 && c.n == n && c.M == M && c.P == P && c.kf == kind_f && c.kb == kind_b &&
        c.radices == radices)
      return i;
  }
  return -1;
}

void spec_shape(int i, int* f64, int* np, int* nt, int* n) {
  *f64 = kSpecs[i].f64;
  *np = kSpecs[i].np;
  *nt = kSpecs[i].nt;
  *n = kSpecs[i].n;
}

// LDS of a specialised kernel: rows of ZP = NP + PAD complex values, n real
// rows or P complex rows, as spec_main_lds in line_pass.h computes it.
size_t spec_lds(int i) {
  const SpecInfo& c = kSpecs[i];
  const size_t es = c.f64 ? 8 : 4;
  const size_t zp = size_t(c.np) + size_t(c.pad);
  const size_t xs = 2 * zp * size_t(c.n);
  const size_t zs = 2 * zp * size_t(c.P);
  const size_t main = ((xs > zs ? xs : zs) * es + 15) / 16 * 16;
  // behind the tile: the lane-ordered Rader constants (spec_ctab_lds), and
  // for fused kernels the axis's eigenvalues when that keeps two workgroups
  // per CU (spec_stage_lam in line_pass.h)
  const size_t ctab = c.rader ? 144 * 2 * es : 0;
  const size_t half = 80 * 1024, lam = size_t(c.n) * es;
  const bool stage = c.kb >= 0 && (main + ctab + lam <= half || main + ctab > half);
  return main + ctab + (stage ? lam : 0);
}

hipError_t launch_spec(int i, const PassArgs& a, hipStream_t s) {
  if (i < 0 || i >= kNumSpecs) return hipErrorInvalidValue;
  return kSpecs[i].launch(a, s, spec_lds(i));
}

// Plane kernel for two axes whose passes have these parameters, or -1.
int find_plane(bool f64, int n, int M, int P, int kind_f, int kind_b, const std::vector<int>& radices) {
  for (int i = 0; i < kNumPlanes; ++i) {
    const PlaneInfo& c = kPlanes[i];
    if ((c.f64 != 0) == f64 && c.n == n && c.M == M && c.P == P && c.kf == kind_f && c.kb == kind_b &&
        c.radices == radices)
      return i;
  }
  return -1;
}

int num_planes() { return kNumPlanes; }

void plane_shape(int i, int* f64, int* nt, int* n) {
  *f64 = kPlanes[i].f64;
  *nt = kPlanes[i].nt;
  *n = kPlanes[i].n;
}

hipError_t launch_plane(int i, const PassArgs& a2, const PassArgs& a1, int inverse, int64_t planes, hipStream_t s) {
  if (i < 0 || i >= kNumPlanes) return hipErrorInvalidValue;
  return kPlanes[i].launch(a2, a1, inverse, planes, s);
}

hipError_t launch_line_pass(int cfg, const PassArgs& a, hipStream_t s) {
  if (cfg < 0 || cfg >= kNum) return hipErrorInvalidValue;
  return kLaunch[cfg](a, s, line_pass_lds(cfg, a.ax.n, a.ax.P));
}

hipError_t launch_line_pass_batch(int cfg, const BatchPassArgs& b, int blocks, size_t lds, hipStream_t s) {
  if (cfg < 0 || cfg >= kNum) return hipErrorInvalidValue;
  return kLaunchBatch[cfg](b, blocks, s, lds);
}

}  // namespace mpois
