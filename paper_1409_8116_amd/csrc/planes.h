// Plane kernels (plane_pass.h): both of the last two axes of a 3D grid in one
// sweep, compiled for one transform that both axes share.
//
// X(ID, type, NT threads, n, M, P, kind of the forward passes, kind of the
// inverse passes, radices...)
// Kinds: 0 R2HC, 1 HC2R (see specs.h).  IDs are consecutive from 0.
#pragma once

#define MPOIS_PLANES(X)                              \
  /* 32 x 32 periodic planes (FP64: 8 x 4 stages, FP32: one radix-32 stage) */ \
  X(0, double, 1024, 32, 32, 32, 0, 1, 8, 4)          \
  X(1, float, 1024, 32, 32, 32, 0, 1, 32)

#define MPOIS_NUM_PLANES 2
