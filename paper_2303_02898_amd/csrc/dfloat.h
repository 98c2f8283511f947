// Double-float arithmetic on FP32 (an unevaluated sum h + l carries about 48
// significant bits): the error-free transformations of Dekker and Knuth (the
// sum by two_sum, the product by one fma), as used for the compensated
// residual passes.  Every function here needs each product and sum rounded on
// its own, so FP contraction is switched off inside them.
#pragma once

#include <hip/hip_runtime.h>

namespace memk {

struct dfl {  // unevaluated sum h + l
  float h, l;
};

__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
  s = a + b;
  const float z = s - a;
  e = (a - (s - z)) + (b - z);
}

// acc += x * y (x, y double-float)
__device__ __forceinline__ void df_acc(dfl& acc, dfl x, dfl y) {
#pragma clang fp contract(off)
  const float p = x.h * y.h;
  const float pe = fmaf(x.h, y.h, -p);
  float sh, se;
  two_sum(acc.h, p, sh, se);
  acc.h = sh;
  acc.l = acc.l + (se + (pe + (x.h * y.l + x.l * y.h)));
}

// acc += x * y (x a plain FP32 value, y double-float): df_acc with x.l = 0
__device__ __forceinline__ void df_acc1(dfl& acc, float x, dfl y) {
#pragma clang fp contract(off)
  const float p = x * y.h;
  const float pe = fmaf(x, y.h, -p);
  float sh, se;
  two_sum(acc.h, p, sh, se);
  acc.h = sh;
  acc.l = acc.l + (se + (pe + x * y.l));
}

// acc += x (x double-float)
__device__ __forceinline__ void df_add(dfl& acc, dfl x) {
#pragma clang fp contract(off)
  float sh, se;
  two_sum(acc.h, x.h, sh, se);
  acc.h = sh;
  acc.l = acc.l + (se + x.l);
}

__device__ __forceinline__ dfl df_norm(dfl a) {
#pragma clang fp contract(off)
  const float h = a.h + a.l;
  return {h, a.l - (h - a.h)};
}

// a + b (b a plain FP32 value), normalised
__device__ __forceinline__ dfl df_plus(dfl a, float b) {
#pragma clang fp contract(off)
  float s, e;
  two_sum(a.h, b, s, e);
  return df_norm({s, e + a.l});
}

// a * b (both double-float), normalised
__device__ __forceinline__ dfl df_mul(dfl a, dfl b) {
#pragma clang fp contract(off)
  const float p = a.h * b.h;
  const float pe = fmaf(a.h, b.h, -p);
  return df_norm({p, pe + (a.h * b.l + a.l * b.h)});
}

// a * b (b a plain FP32 value), normalised
__device__ __forceinline__ dfl df_mul1(dfl a, float b) {
#pragma clang fp contract(off)
  const float p = a.h * b;
  const float pe = fmaf(a.h, b, -p);
  return df_norm({p, pe + a.l * b});
}

// 1 / a for a plain FP32 value a: the quotient and its remainder term
__device__ __forceinline__ dfl df_recip(float a) {
  const float h = 1.f / a;
  return {h, fmaf(-a, h, 1.f) * h};
}

}  // namespace memk
