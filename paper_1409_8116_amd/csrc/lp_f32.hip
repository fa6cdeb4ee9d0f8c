// FP32 instantiations of the line-transform kernel.
#include "cfgs.h"
#include "line_pass.h"

namespace mpois {

hipError_t launch_line_pass_f32(int i, const PassArgs& a, hipStream_t s, size_t lds) {
  int idx = 0;
#define X(T, NP, NT, PMAX) \
  if (idx++ == i) return launch_lp<T, NP, NT, PMAX>(a, s, lds);
  MPOIS_CFGS_F32(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_line_pass_batch_f32(int i, const BatchPassArgs& b, int blocks, hipStream_t s, size_t lds) {
  int idx = 0;
#define X(T, NP, NT, PMAX) \
  if (idx++ == i) return launch_lp_batch<T, NP, NT, PMAX>(b, blocks, s, lds);
  MPOIS_CFGS_F32(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t prepare_line_pass_f32() {
  hipError_t e = hipSuccess;
#define X(T, NP, NT, PMAX) \
  if (e == hipSuccess) e = prepare_lp<T, NP, NT, PMAX>();
  MPOIS_CFGS_F32(X)
#undef X
  return e;
}

}  // namespace mpois
