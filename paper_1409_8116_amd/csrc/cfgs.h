// Instantiated shapes of the line-transform kernel: (ID, type, NP line pairs
// per tile, NT threads, PMAX longest DFT work length, RADER: 1 if the prime-73
// Rader stage is compiled in).  IDs are consecutive from 0.
#pragma once

#define MPOIS_CFGS_F64(X)      \
  X(0, double, 8, 512, 1024, 0)   \
  X(1, double, 8, 256, 1024, 1)   \
  X(2, double, 4, 256, 1024, 1)   \
  X(3, double, 4, 512, 2048, 0)   \
  X(4, double, 2, 512, 4096, 0)   \
  X(5, double, 1, 512, 8192, 0)

#define MPOIS_CFGS_F32(X)      \
  X(6, float, 16, 512, 1024, 1)   \
  X(7, float, 8, 256, 1024, 1)    \
  X(8, float, 8, 512, 2048, 0)    \
  X(9, float, 4, 512, 4096, 0)    \
  X(10, float, 2, 512, 8192, 0)

#define MPOIS_CFGS(X) MPOIS_CFGS_F64(X) MPOIS_CFGS_F32(X)
