// Kernels specialised for the transforms of the hot workloads: everything
// about the line transform is a compile-time constant (line length, DFT and
// work length, kinds, Stockham stages), so index arithmetic folds and loops
// have exact trip counts.  The plan uses one when a pass's description
// matches it exactly (same kinds, lengths and radix list), else the generic
// line_pass shapes of cfgs.h.
//
// X(ID, type, NP line pairs per tile, NT threads, RADER lanes (0: none, 1),
//   SLIM, PAD, n, M, P, kind_f, kind_b (-1: none), radices...)
// PAD: complex values of padding per LDS row (row pitch NP + PAD).
// Kinds: 0 R2HC, 1 HC2R, 2 DCT-II, 3 DCT-III, 4 DST-II, 5 DST-III, 6 DCT-I, 7 DST-I.
// IDs are consecutive from 0.
#pragma once

#define MPOIS_SPECS(X)                                            \
  /* 512-point DCT-I (vertex Neumann, 1022 = 73 x 14) */          \
  X(0, float, 8, 256, 2, 0, 1, 512, 1022, 1022, 6, -1, 73, 14)       \
  X(1, float, 8, 256, 2, 0, 0, 512, 1022, 1022, 6, 6, 73, 14)        \
  X(2, double, 4, 256, 4, 0, 0, 512, 1022, 1022, 6, -1, 73, 14)      \
  X(3, double, 4, 256, 4, 0, 0, 512, 1022, 1022, 6, 6, 73, 14)       \
  /* 256-point periodic / staggered Dirichlet / staggered Neumann */ \
  X(4, double, 8, 512, 0, 1, 1, 256, 256, 256, 2, -1, 16, 16)        \
  X(5, double, 8, 512, 0, 1, 1, 256, 256, 256, 4, -1, 16, 16)        \
  X(6, double, 8, 512, 0, 1, 1, 256, 256, 256, 0, 1, 16, 16)         \
  X(7, double, 8, 512, 0, 1, 1, 256, 256, 256, 5, -1, 16, 16)        \
  X(8, double, 8, 512, 0, 1, 1, 256, 256, 256, 3, -1, 16, 16)        \
  X(9, float, 8, 512, 0, 1, 1, 256, 256, 256, 2, -1, 16, 16)         \
  X(10, float, 8, 512, 0, 1, 1, 256, 256, 256, 4, -1, 16, 16)        \
  X(11, float, 8, 512, 0, 1, 1, 256, 256, 256, 0, 1, 16, 16)         \
  X(12, float, 8, 512, 0, 1, 1, 256, 256, 256, 5, -1, 16, 16)        \
  X(13, float, 8, 512, 0, 1, 1, 256, 256, 256, 3, -1, 16, 16)        \
  /* channel: 256-point periodic, 512-point staggered Neumann, 1024-point periodic */ \
  X(14, float, 8, 512, 0, 1, 1, 256, 256, 256, 0, -1, 16, 16)        \
  X(15, float, 8, 512, 0, 1, 1, 256, 256, 256, 1, -1, 16, 16)        \
  X(16, float, 16, 512, 0, 1, 1, 512, 512, 512, 2, -1, 32, 16)        \
  X(17, float, 16, 512, 0, 1, 1, 512, 512, 512, 3, -1, 32, 16)        \
  X(18, float, 8, 512, 0, 1, 1, 1024, 1024, 1024, 0, 1, 32, 32)      \
  /* 32-point periodic (FP64) */                                   \
  X(19, double, 8, 512, 0, 1, 1, 32, 32, 32, 0, -1, 8, 4)            \
  X(20, double, 8, 512, 0, 1, 1, 32, 32, 32, 0, 1, 8, 4)             \
  X(21, double, 8, 512, 0, 1, 1, 32, 32, 32, 1, -1, 8, 4)            \
  /* channel in FP64 (the projection step's FP64 plans) */         \
  X(22, double, 8, 512, 0, 1, 1, 256, 256, 256, 0, -1, 16, 16)       \
  X(23, double, 8, 512, 0, 1, 1, 256, 256, 256, 1, -1, 16, 16)       \
  X(24, double, 8, 512, 0, 1, 1, 512, 512, 512, 2, -1, 8, 8, 8)      \
  X(25, double, 8, 512, 0, 1, 1, 512, 512, 512, 3, -1, 8, 8, 8)      \
  X(26, double, 4, 512, 0, 1, 0, 1024, 1024, 1024, 0, 1, 16, 8, 8)

#define MPOIS_NUM_SPECS 27
