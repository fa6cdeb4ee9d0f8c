// Instantiated shapes of the line-transform kernel: (type, NP pairs per tile,
// NT threads, PMAX longest DFT work length).  Index order = FP64 list, then FP32.
#pragma once

#define MPOIS_CFGS_F64(X)   \
  X(double, 8, 512, 1024)   \
  X(double, 4, 256, 1024)   \
  X(double, 4, 512, 2048)   \
  X(double, 2, 512, 4096)   \
  X(double, 1, 512, 8192)

#define MPOIS_CFGS_F32(X)   \
  X(float, 16, 512, 1024)   \
  X(float, 8, 256, 1024)    \
  X(float, 8, 512, 2048)    \
  X(float, 4, 512, 4096)    \
  X(float, 2, 512, 8192)
