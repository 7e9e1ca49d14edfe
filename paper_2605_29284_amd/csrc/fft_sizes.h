// Transform lengths F = N1 * N2 compiled into the library (even 2^a 3^b ladder).
// Any length >= the linear-convolution bound gives the same result up to rounding,
// so the plan picks the smallest listed length that is large enough.
#pragma once
#define KRIG_FFT_SIZES(X)                                                                      \
  X(4, 4) X(6, 4) X(8, 4) X(6, 6) X(8, 6) X(8, 8) X(9, 8) X(12, 8) X(16, 8) X(12, 12) X(16, 12) \
  X(16, 16) X(18, 16) X(24, 16) X(32, 16) X(24, 24) X(32, 24) X(36, 24) X(32, 32) X(36, 32)    \
  X(48, 32) X(64, 32) X(48, 48) X(64, 48)
