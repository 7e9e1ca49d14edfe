// Transform lengths F = R1 * R2 * R3 compiled into the library (even 2^a 3^b
// ladder).  Any length >= the linear-convolution bound gives the same result up to
// rounding, so the plan picks the smallest listed length that is large enough.
// Up to 288 the transforms are two-stage (R1 = 1); longer ones add an outer radix-8
// or radix-16 pass so that a thread holds at most 16 values (18 at length 288).
#pragma once
#define KRIG_FFT_SIZES(X)                                                                     \
  X(1, 4, 4) X(1, 6, 4) X(1, 8, 4) X(1, 6, 6) X(1, 8, 6) X(1, 8, 8) X(1, 9, 8) X(1, 12, 8)    \
  X(1, 16, 8) X(1, 12, 12) X(1, 16, 12) X(1, 16, 16) X(1, 18, 16) X(8, 8, 6) X(8, 8, 8)      \
  X(8, 9, 8) X(8, 12, 8) X(8, 12, 9) X(8, 16, 8) X(8, 12, 12) X(8, 16, 12) X(16, 16, 8)      \
  X(16, 12, 12) X(16, 16, 12)

// Further factorisations of some lengths, compiled as well: the default (first) form
// of each length comes from the list above; krig_plan_tune / krig_plan_autotune may
// switch a plan's row or column transforms to one of these.
#define KRIG_FFT_VARIANTS(X)                                                                  \
  X(1, 24, 16) X(1, 32, 16) X(1, 24, 24) X(12, 8, 8) X(8, 8, 12) X(1, 32, 24) X(1, 36, 24)   \
  X(16, 8, 8) X(12, 12, 8) X(1, 36, 32) X(12, 16, 12)
