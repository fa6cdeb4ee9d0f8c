// Instantiated shapes of the line-transform kernel: (ID, type, NP line pairs
// per tile, NT threads, PMAX longest DFT work length, RADER: 0, or the
// number of lanes (2, 4 or 8) per butterfly of the compiled-in prime-73 Rader stage, SLIM: 1 for shapes compiled for 4 waves per SIMD
// (two 512-thread workgroups per CU) without the radix-11/13 codelets, 2 for
// the wide shapes that also carry the prime codelets 17, 19, 23, 29 and 31
// (their registers would lower every other shape's occupancy)).
// IDs are consecutive from 0.
#pragma once

#define MPOIS_CFGS_F64(X)          \
  X(0, double, 8, 512, 1024, 0, 1)  \
  X(1, double, 8, 512, 1024, 4, 0)  \
  X(2, double, 4, 256, 1024, 4, 0)  \
  X(3, double, 4, 512, 2048, 0, 1)  \
  X(4, double, 2, 512, 4096, 0, 1)  \
  X(5, double, 1, 512, 8192, 0, 1)  \
  X(6, double, 8, 512, 1024, 0, 0)  \
  X(7, double, 4, 512, 4096, 0, 0)

#define MPOIS_CFGS_F32(X)          \
  X(8, float, 16, 512, 1024, 2, 0)  \
  X(9, float, 8, 256, 1024, 2, 0)   \
  X(10, float, 8, 512, 2048, 0, 1)  \
  X(11, float, 4, 512, 4096, 0, 1)  \
  X(12, float, 2, 512, 8192, 0, 1)  \
  X(13, float, 8, 512, 1024, 0, 1)  \
  X(14, float, 16, 512, 1024, 0, 0) \
  X(15, float, 4, 512, 4096, 0, 0)  \
  X(16, double, 2, 512, 2048, 0, 2) \
  X(17, float, 2, 256, 2048, 0, 2)

#define MPOIS_CFGS(X) MPOIS_CFGS_F64(X) MPOIS_CFGS_F32(X)
#define MPOIS_NUM_CFGS 18
