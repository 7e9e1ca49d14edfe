// Storage forms of the half spectra that pass between the transform kernels.
//
// The transforms compute in registers (FP64 for the prediction and its adjoint); what
// a pass writes for the next one may be stored narrower: cx<double> (16 bytes per
// complex value) or cx<float> (8 bytes, one FP32 rounding, relative 2^-24).  Which
// spectrum takes which form is the plan's choice (spec_bytes in plan.cpp).
//
// Spec<TS> is a pointer into one field's block with element-wise load and store (the
// arithmetic type TC is converted on the way); field(base, fs, b) addresses field b of
// a buffer whose fields hold fs elements each.
#pragma once
#include "krig_internal.h"

namespace krig {

template <typename TS> struct Spec {
  cx<TS>* p;
  using raw = cx<TS>;
  static __device__ __forceinline__ Spec field(const void* base, int64_t fs, int64_t b) {
    return Spec{const_cast<cx<TS>*>(reinterpret_cast<const cx<TS>*>(base)) + b * fs};
  }
  __device__ __forceinline__ Spec at(int64_t i) const { return Spec{p + i}; }
  __device__ __forceinline__ raw ldraw(int64_t i) const { return p[i]; }
  static __device__ __forceinline__ raw zero() { return mk<TS>(0, 0); }
  template <typename TC> static __device__ __forceinline__ cx<TC> cvt(raw r) { return ccast<TC>(r); }
  template <typename TC> __device__ __forceinline__ cx<TC> ld(int64_t i) const { return ccast<TC>(p[i]); }
  template <typename TC> __device__ __forceinline__ void st(int64_t i, cx<TC> v) const { p[i] = ccast<TS>(v); }
};

// Storage forms of one column pass: its input, second input (lag-gradient pass: the
// saved spectra of c*), output and partial lag-gradient spectra.
template <typename IN, typename IN2, typename OUT, typename PART> struct Stor {
  using in = IN;
  using in2 = IN2;
  using out = OUT;
  using part = PART;
};

}  // namespace krig
