// Small in-register FFTs shared by the FFT fine form and the
// frequency-domain mGIFT (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

namespace fftreg {

// Complex product with its fused multiply-adds written out, so that the
// rounding does not depend on how the compiler contracts the surrounding code.
__device__ inline float2 cmulf(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}

__host__ __device__ constexpr int bitrev(int i, int n) {
  int r = 0;
  for (int s = 1; s < n; s <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// exp(+j 2 pi k / 64) for k < 64, evaluated at compile time (Taylor series
// of sin and cos on [-pi, pi], 24 terms: truncation far below double
// rounding), so that twiddle factors of the unrolled FFTs fold into
// instruction constants.
struct Tw64 {
  float re[64], im[64];
};

constexpr double kPi = 3.14159265358979323846;

constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 24; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}

constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 24; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

constexpr Tw64 make_tw64() {
  Tw64 t{};
  for (int k = 0; k < 64; ++k) {
    double a = 2.0 * kPi * k / 64.0;
    if (a > kPi) a -= 2.0 * kPi;
    t.re[k] = (float)taylor_cos(a);
    t.im[k] = (float)taylor_sin(a);
  }
  return t;
}

__device__ constexpr Tw64 kTw = make_tw64();
static_assert(make_tw64().re[0] == 1.0f && make_tw64().im[16] == 1.0f &&
                  make_tw64().re[32] == -1.0f,
              "twiddle table");

// x * exp(+j 2 pi idx / 64), idx a compile-time constant after unrolling:
// the factors 1, j, -j and exp(+-j pi/4), exp(+-j 3pi/4) take adds and one
// multiply instead of a full complex product (IEEE rules keep the compiler
// from dropping products by the zero parts itself).
__device__ inline float2 twiddle(float2 x, int idx) {
  constexpr float h = 0.70710678118654752f;  // sqrt(1/2)
  switch (idx) {
    case 0: return x;
    case 16: return make_float2(-x.y, x.x);
    case 48: return make_float2(x.y, -x.x);
    case 8: return make_float2(h * (x.x - x.y), h * (x.x + x.y));
    case 24: return make_float2(-h * (x.x + x.y), h * (x.x - x.y));
    case 40: return make_float2(h * (x.y - x.x), -h * (x.x + x.y));
    case 56: return make_float2(h * (x.x + x.y), h * (x.y - x.x));
    default: return cmulf(x, make_float2(kTw.re[idx], kTw.im[idx]));
  }
}

// Butterfly a +- x exp(+j 2 pi idx / 64).  For the factors exp(+-j pi/4),
// exp(+-j 3pi/4) the scaling by sqrt(1/2) is fused into the additions; every
// fused operation is written out (fmaf), none is left to the compiler.
__device__ inline void butterfly(float2 &a, float2 &x, int idx) {
  constexpr float h = 0.70710678118654752f;  // sqrt(1/2)
  float s1, s2, c1, c2;                       // b = (c1 h s1, c2 h s2)
  switch (idx) {
    case 8: s1 = x.x - x.y; s2 = x.x + x.y; c1 = h; c2 = h; break;
    case 24: s1 = x.x + x.y; s2 = x.x - x.y; c1 = -h; c2 = h; break;
    case 40: s1 = x.y - x.x; s2 = x.x + x.y; c1 = h; c2 = -h; break;
    case 56: s1 = x.x + x.y; s2 = x.y - x.x; c1 = h; c2 = h; break;
    default: {
      const float2 b = twiddle(x, idx);
      const float2 t = a;
      a = make_float2(t.x + b.x, t.y + b.y);
      x = make_float2(t.x - b.x, t.y - b.y);
      return;
    }
  }
  const float2 t = a;
  a = make_float2(fmaf(c1, s1, t.x), fmaf(c2, s2, t.y));
  x = make_float2(fmaf(-c1, s1, t.x), fmaf(-c2, s2, t.y));
}

// In-register radix-2 FFT, N a power of two <= 64, positive exponent:
// x[k] <- sum_j x[j] exp(+j 2 pi j k / N), natural order in and out.
template <int N>
__device__ inline void fft_reg(float2 (&x)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int j = bitrev(i, N);
    if (j > i) {
      const float2 t = x[i];
      x[i] = x[j];
      x[j] = t;
    }
  }
#pragma unroll
  for (int len = 2; len <= N; len <<= 1) {
#pragma unroll
    for (int i = 0; i < N; i += len) {
#pragma unroll
      for (int k = 0; k < len / 2; ++k) butterfly(x[i + k], x[i + k + len / 2], k * (64 / len));
    }
  }
}

}  // namespace fftreg
