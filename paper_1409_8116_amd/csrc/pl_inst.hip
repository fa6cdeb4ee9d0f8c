// The plane kernels of planes.h (one object for all: they are small).
#include "plane_pass.h"
#include "planes.h"

namespace mpois {

#define X(ID, T, NT, N, M, P, KF, KB, ...)                                                              \
  hipError_t launch_plane_##ID(const PassArgs& a2, const PassArgs& a1, int inverse, int64_t planes,  \
                               hipStream_t s) {                                                      \
    return launch_plane_t<T, NT, N, M, P, KF, KB, __VA_ARGS__>(a2, a1, inverse, planes, s);           \
  }
MPOIS_PLANES(X)
#undef X

}  // namespace mpois
