// Kernel-shape table and dispatch of the line-transform kernel.
#include <hip/hip_runtime.h>

#include "cfgs.h"
#include "internal.h"

namespace mpois {

// one set per shape, defined in lp_inst.hip compiled with MPOIS_CFG = shape id
#define MPOIS_DECL(I)                                                                                      \
  hipError_t launch_line_pass_cfg##I(const PassArgs& a, hipStream_t s, size_t lds);                        \
  hipError_t launch_line_pass_batch_cfg##I(const BatchPassArgs& b, int blocks, hipStream_t s, size_t lds); \
  hipError_t prepare_line_pass_cfg##I();
MPOIS_DECL(0) MPOIS_DECL(1) MPOIS_DECL(2) MPOIS_DECL(3) MPOIS_DECL(4) MPOIS_DECL(5) MPOIS_DECL(6)
MPOIS_DECL(7) MPOIS_DECL(8) MPOIS_DECL(9) MPOIS_DECL(10) MPOIS_DECL(11) MPOIS_DECL(12) MPOIS_DECL(13)
MPOIS_DECL(14) MPOIS_DECL(15)
#undef MPOIS_DECL

namespace {
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
static_assert(kNum == 16, "update the per-shape function tables below");

using LaunchFn = hipError_t (*)(const PassArgs&, hipStream_t, size_t);
using LaunchBatchFn = hipError_t (*)(const BatchPassArgs&, int, hipStream_t, size_t);
using PrepareFn = hipError_t (*)();
#define MPOIS_ROW(F) \
  F##0, F##1, F##2, F##3, F##4, F##5, F##6, F##7, F##8, F##9, F##10, F##11, F##12, F##13, F##14, F##15
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
  return hipSuccess;
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
