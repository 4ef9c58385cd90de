// Stockham autosort FFT of a power-of-two length NP held in LDS, one
// workgroup of 256 threads per transform.  The pass with span NS and radix R
// reads X[j + t NP/R], scales by W^(t (j mod NS)), runs an R-point FFT in
// registers and writes X[(j/NS) NS R + (j mod NS) + t NS].  Every thread loads
// all its groups before the barrier and writes after it, so the pass works in
// place.  The radices are 16 with the remainder folded into the first pass (32
// or 64) or a last pass of 4 or 8, so NP = 8192 takes three passes.  Twiddles
// come from two small LDS tables, W^i = TH[i >> 7] TL[i & 127].  Element i
// sits at LDS index i + i / 32 (one pad entry per 32): the span-1 pass writes
// with a stride of R entries, which would otherwise put every lane of a
// wavefront in the same bank; contiguous accesses stay contiguous.
#pragma once

#include "fft_reg.h"

namespace fftlds {

using fftreg::cmulf;
using fftreg::fft_reg;

__device__ inline float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

// Padded LDS position of element i, and the LDS entries an NP-point transform
// occupies.
__device__ inline int pidx(int i) { return i + (i >> 5); }
template <int NP>
constexpr int lds_len() { return NP + NP / 32; }

// Twiddle W^i = exp(+j 2 pi i / NP) from the two LDS tables.
struct TwLds {
  const float2 *lo;  // [128] W^i
  const float2 *hi;  // [NP / 128] W^(128 i)
  __device__ float2 operator()(int i) const { return cmulf(hi[i >> 7], lo[i & 127]); }
};

// One Stockham pass; INV selects the sign.
template <int NP, int NS, int R, bool INV>
__device__ inline void stockham_pass(float2 *X, const TwLds &tw) {
  constexpr int NG = NP / R;
  constexpr int GPT = (NG + 255) / 256;
  const int tid = threadIdx.x;
  float2 v[GPT][R];
#pragma unroll
  for (int g = 0; g < GPT; ++g) {
    const int j = tid + 256 * g;
    if (j < NG) {
      const int k = j % NS;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        float2 x = X[pidx(j + t * NG)];
        if (NS > 1 && t > 0) {
          const float2 w = tw(t * k * (NP / (NS * R)));
          x = cmulf(x, INV ? w : conjf2(w));
        }
        v[g][t] = x;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < GPT; ++g) {
    const int j = tid + 256 * g;
    if (j < NG) {
      const int k = j % NS;
      if (!INV) {
#pragma unroll
        for (int t = 0; t < R; ++t) v[g][t] = conjf2(v[g][t]);
      }
      fft_reg<R>(v[g]);
      const int d = (j / NS) * NS * R + k;
#pragma unroll
      for (int t = 0; t < R; ++t) X[pidx(d + t * NS)] = INV ? v[g][t] : conjf2(v[g][t]);
    }
  }
  __syncthreads();
}

// Radix of the pass with span NS: NP = 16^q r; r = 2 (or 4 for NP >= 16384)
// joins the first pass (32, 64), otherwise r is a last pass (4, 8).
template <int NP, int NS>
constexpr int pass_radix() {
  int e = 0;
  while ((1 << e) < NP) ++e;
  const int rem = e % 4;
  if (NS == 1 && e >= 5 && (rem == 1 || (rem == 2 && NP >= 16384))) return 16 << rem;
  const int left = NP / NS;
  return left % 16 == 0 ? 16 : left;
}

template <int NP, int NS, bool INV>
__device__ inline void fft_lds(float2 *X, const TwLds &tw) {
  if constexpr (NS < NP) {
    constexpr int R = pass_radix<NP, NS>();
    static_assert(NP % (NS * R) == 0, "radix plan");
    stockham_pass<NP, NS, R, INV>(X, tw);
    fft_lds<NP, NS * R, INV>(X, tw);
  }
}

// Fill the two twiddle tables from the global W table.
template <int NP>
__device__ inline TwLds load_twiddles(const float2 *__restrict__ tw, float2 *lo, float2 *hi) {
  constexpr int NH = NP / 128 > 1 ? NP / 128 : 1;
  for (int i = threadIdx.x; i < 128 + NH; i += 256) {
    if (i < 128) lo[i] = tw[i % NP];
    else hi[i - 128] = tw[((i - 128) * 128) % NP];
  }
  return TwLds{lo, hi};
}

}  // namespace fftlds
