#include "tune.h"

#include "mpois.h"

namespace mpois {
bool tune_enabled(unsigned flags) { return (flags & MPOIS_FLAG_TUNE) != 0; }
int tuned_cfg(int fallback, bool, int, int, bool) { return fallback; }
}  // namespace mpois
