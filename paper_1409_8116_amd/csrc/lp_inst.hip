// One instantiation of the line-transform kernel, selected at build time by
// MPOIS_CFG (an index into the shape list of cfgs.h); the build compiles this
// file once per shape so that the shapes build in parallel.
#include "cfgs.h"
#include "line_pass.h"

#ifndef MPOIS_CFG
#error "MPOIS_CFG must be defined"
#endif

namespace mpois {

#define MPOIS_PASTE2(a, b) a##b
#define MPOIS_PASTE(a, b) MPOIS_PASTE2(a, b)

hipError_t MPOIS_PASTE(launch_line_pass_cfg, MPOIS_CFG)(const PassArgs& a, hipStream_t s, size_t lds) {
#define X(ID, T, NP, NT, PMAX, RADER, SLIM) \
  if constexpr (ID == MPOIS_CFG) return launch_lp<T, NP, NT, PMAX, RADER, SLIM>(a, s, lds);
  MPOIS_CFGS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t MPOIS_PASTE(launch_line_pass_batch_cfg, MPOIS_CFG)(const BatchPassArgs& b, int blocks, hipStream_t s,
                                                             size_t lds) {
#define X(ID, T, NP, NT, PMAX, RADER, SLIM) \
  if constexpr (ID == MPOIS_CFG) return launch_lp_batch<T, NP, NT, PMAX, RADER, SLIM>(b, blocks, s, lds);
  MPOIS_CFGS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t MPOIS_PASTE(prepare_line_pass_cfg, MPOIS_CFG)() {
#define X(ID, T, NP, NT, PMAX, RADER, SLIM) \
  if constexpr (ID == MPOIS_CFG) return prepare_lp<T, NP, NT, PMAX, RADER, SLIM>();
  MPOIS_CFGS(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace mpois
