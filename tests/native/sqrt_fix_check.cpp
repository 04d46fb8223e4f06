// Exhaustive host check of the kernels' square-root rounding correction
// (sqrt_round_fix in the library's sqrt_fix.h, included verbatim): for every
// float x in [2^-96, FLT_MAX] and every s one float below, at, and one float
// above the correctly rounded root r = sqrtf(x) (the host's IEEE square root),
// sqrt_round_fix(x, s) must return r; and for x = +0 it must return +0.  A hardware root within one ulp of the
// exact root is always one of these three floats, so this proves the kernels'
// fast root equal to sqrtf over that range, whatever the hardware's exact error.
//
// Built by the test with g++ -O2 -mfma -fopenmp; prints the count checked and
// the first failure, exits non-zero on any failure.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#define __host__
#define __device__
#include "sqrt_fix.h"

static float from_bits(uint32_t u) {
  float f;
  memcpy(&f, &u, sizeof f);
  return f;
}
static uint32_t to_bits(float f) {
  uint32_t u;
  memcpy(&u, &f, sizeof u);
  return u;
}

int main() {
  const uint32_t first = to_bits(0x1p-96f);
  const uint32_t last = to_bits(3.40282347e38f);  // FLT_MAX
  long long checked = 0, bad = 0;
  uint32_t bad_x = 0;
  int bad_k = 0;
#pragma omp parallel for schedule(dynamic, 1 << 16) reduction(+ : checked, bad)
  for (long long u = first; u <= (long long)last; ++u) {
    const float x = from_bits((uint32_t)u);
    const float r = sqrtf(x);
    const uint32_t rb = to_bits(r);
    for (int k = -1; k <= 1; ++k) {
      const float s = from_bits(rb + (uint32_t)k);
      ++checked;
      if (to_bits(sqrt_round_fix(x, s)) != rb) {
        ++bad;
#pragma omp critical
        {
          bad_x = (uint32_t)u;
          bad_k = k;
        }
      }
    }
  }
  // x = +0 (lambda 1 where all channels of two pixels are equal): the root is
  // +0, for s = +0 and for s one float above it
  for (uint32_t sb = 0; sb <= 1; ++sb) {
    ++checked;
    if (to_bits(sqrt_round_fix(0.0f, from_bits(sb))) != 0u) {
      ++bad;
      bad_x = 0u;
      bad_k = (int)sb;
    }
  }
  printf("checked %lld (x, s) pairs over [2^-96, FLT_MAX] and x = +0; failures %lld\n", checked, bad);
  if (bad) printf("e.g. x = %a (bits 0x%08x), s = r %+d ulp\n", from_bits(bad_x), bad_x, bad_k);
  return bad ? 1 : 0;
}
