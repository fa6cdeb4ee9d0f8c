// Kernel-shape autotuner interface (tile width / work length per line pass).
#pragma once

namespace mpois {
bool tune_enabled(unsigned flags);
// Best kernel configuration for a line pass of length-n lines whose DFT work
// length is P; `fallback` is returned when nothing better is known.
int tuned_cfg(int fallback, bool f64, int n, int P, bool contiguous);
}  // namespace mpois
