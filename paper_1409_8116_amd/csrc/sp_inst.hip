// One specialised line-transform kernel, selected at build time by MPOIS_SPEC
// (an index into the list of specs.h); the build compiles this file once per
// entry so that they build in parallel.
#include "line_pass.h"
#include "specs.h"

#ifndef MPOIS_SPEC
#error "MPOIS_SPEC must be defined"
#endif

namespace mpois {

#define MPOIS_PASTE2(a, b) a##b
#define MPOIS_PASTE(a, b) MPOIS_PASTE2(a, b)

hipError_t MPOIS_PASTE(launch_spec_, MPOIS_SPEC)(const PassArgs& a, hipStream_t s, size_t lds) {
#define X(ID, T, NP, NT, RADER, SLIM, PAD, N, M, P, KF, KB, ...) \
  if constexpr (ID == MPOIS_SPEC) return launch_spec_t<T, NP, NT, RADER, SLIM, PAD, N, M, P, KF, KB, __VA_ARGS__>(a, s, lds);
  MPOIS_SPECS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t MPOIS_PASTE(prepare_spec_, MPOIS_SPEC)() {
#define X(ID, T, NP, NT, RADER, SLIM, PAD, N, M, P, KF, KB, ...) \
  if constexpr (ID == MPOIS_SPEC) return prepare_spec_t<T, NP, NT, RADER, SLIM, PAD, N, M, P, KF, KB, __VA_ARGS__>();
  MPOIS_SPECS(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace mpois
