// Rounding correction of a square root: given x in [2^-96, FLT_MAX] and s, a
// float within one ulp of sqrt(x), return the correctly rounded sqrtf(x); for
// x = +0 (with s = +0 or the next float) it returns +0.
//
// This is the Tuckerman rounding test, in the form Markstein gives for fused
// multiply-add hardware: with lo and hi the floats next to s, the residuals
// x - lo * s and x - hi * s, each computed with a single rounding by an fma,
// tell on which side of the midpoints (lo + s) / 2 and (s + hi) / 2 the exact
// root lies, up to a term below half an ulp that cannot change the sign.  The
// whole range has been checked exhaustively on the host for s one float below,
// at and above the correctly rounded root.
#pragma once

__host__ __device__ inline float sqrt_round_fix(float x, float s) {
  const float lo = __builtin_bit_cast(float, __builtin_bit_cast(int, s) - 1);
  const float hi = __builtin_bit_cast(float, __builtin_bit_cast(int, s) + 1);
  const float e_lo = fmaf(-lo, s, x);
  const float e_hi = fmaf(-hi, s, x);
  float r = e_lo <= 0.0f ? lo : s;
  r = e_hi > 0.0f ? hi : r;
  return r;
}
