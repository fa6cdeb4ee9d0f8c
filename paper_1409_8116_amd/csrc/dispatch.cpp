// Kernel-shape table and dispatch of the line-transform kernel.
#include <hip/hip_runtime.h>

#include "cfgs.h"
#include "internal.h"

namespace mpois {

hipError_t launch_line_pass_f64(int i, const PassArgs& a, hipStream_t s, size_t lds);
hipError_t launch_line_pass_f32(int i, const PassArgs& a, hipStream_t s, size_t lds);
hipError_t launch_line_pass_batch_f64(int i, const BatchPassArgs& b, int blocks, hipStream_t s, size_t lds);
hipError_t launch_line_pass_batch_f32(int i, const BatchPassArgs& b, int blocks, hipStream_t s, size_t lds);
hipError_t prepare_line_pass_f64();
hipError_t prepare_line_pass_f32();

namespace {
struct KernelCfg {
  int f64, np, nt, pmax;
};
const KernelCfg kCfgs[] = {
#define X(T, NP, NT, PMAX) {sizeof(T) == 8, NP, NT, PMAX},
    MPOIS_CFGS_F64(X) MPOIS_CFGS_F32(X)
#undef X
};
constexpr int kNumF64 = 0
#define X(T, NP, NT, PMAX) +1
    MPOIS_CFGS_F64(X)
#undef X
    ;
}  // namespace

int num_kernel_cfgs() { return int(sizeof(kCfgs) / sizeof(kCfgs[0])); }

void kernel_cfg(int i, int* f64, int* np, int* nt, int* pmax) {
  *f64 = kCfgs[i].f64;
  *np = kCfgs[i].np;
  *nt = kCfgs[i].nt;
  *pmax = kCfgs[i].pmax;
}

// LDS bytes: the larger of the real tile (2 NP rows, odd pitch) and the
// complex work buffer (NP pairs of P values).
size_t line_pass_lds(int cfg, int n, int P) {
  const KernelCfg& c = kCfgs[cfg];
  const size_t es = c.f64 ? 8 : 4;
  const size_t tl = 2 * size_t(c.np);
  const size_t xs = tl * size_t((n | 1) + 1);
  const size_t zs = 2 * size_t(c.np) * size_t(P);
  return (xs > zs ? xs : zs) * es;
}

hipError_t prepare_kernels() {
  hipError_t e = prepare_line_pass_f64();
  if (e == hipSuccess) e = prepare_line_pass_f32();
  return e;
}

hipError_t launch_line_pass(int cfg, const PassArgs& a, hipStream_t s) {
  if (cfg < 0 || cfg >= num_kernel_cfgs()) return hipErrorInvalidValue;
  const size_t lds = line_pass_lds(cfg, a.ax.n, a.ax.P);
  return cfg < kNumF64 ? launch_line_pass_f64(cfg, a, s, lds) : launch_line_pass_f32(cfg - kNumF64, a, s, lds);
}

hipError_t launch_line_pass_batch(int cfg, const BatchPassArgs& b, int blocks, size_t lds, hipStream_t s) {
  if (cfg < 0 || cfg >= num_kernel_cfgs()) return hipErrorInvalidValue;
  return cfg < kNumF64 ? launch_line_pass_batch_f64(cfg, b, blocks, s, lds)
                       : launch_line_pass_batch_f32(cfg - kNumF64, b, blocks, s, lds);
}

}  // namespace mpois
