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
//
// fft_lds_io runs the same passes on input the caller holds in registers:
// the first pass (span 1, no twiddles) works on those registers and the last
// pass hands its results to a callback, so the transform makes two LDS round
// trips and two barriers fewer than a fill of X, fft_lds and a read-out, with
// the same arithmetic (bit-identical results).
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
constexpr int radix_at(int np, int ns) {
  int e = 0;
  while ((1 << e) < np) ++e;
  const int rem = e % 4;
  if (ns == 1 && e >= 5 && (rem == 1 || (rem == 2 && np >= 16384))) return 16 << rem;
  const int left = np / ns;
  return left % 16 == 0 ? 16 : left;
}
template <int NP, int NS>
constexpr int pass_radix() { return radix_at(NP, NS); }

// Span of the last pass (the one whose span times radix is NP).
constexpr int last_span(int np) {
  int ns = 1;
  while (ns * radix_at(np, ns) < np) ns *= radix_at(np, ns);
  return ns;
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

// The passes with spans from NS up to (not including) NS_END.
template <int NP, int NS, int NS_END, bool INV>
__device__ inline void fft_lds_span(float2 *X, const TwLds &tw) {
  if constexpr (NS < NS_END) {
    constexpr int R = pass_radix<NP, NS>();
    stockham_pass<NP, NS, R, INV>(X, tw);
    fft_lds_span<NP, NS * R, NS_END, INV>(X, tw);
  }
}

// Radix of the first pass: fft_lds_io's v holds that many elements.
template <int NP>
constexpr int first_radix() { return radix_at(NP, 1); }

// Transform of NP elements given in registers: thread j < NP / R1 (R1 =
// first_radix<NP>()) holds element j + t NP / R1 in v[t]; other threads'
// v is not read.  Each output element i is passed once to store(i, value)
// by one thread.  X is the LDS work area (lds_len<NP>() entries); every
// thread of the workgroup must call this.
template <int NP, bool INV, class Store>
__device__ inline void fft_lds_io(float2 (&v)[first_radix<NP>()], float2 *X, const TwLds &tw,
                                  Store store) {
  constexpr int R1 = first_radix<NP>(), NG1 = NP / R1, LS = last_span(NP), RL = NP / LS;
  static_assert(NG1 <= 256 && R1 < NP && LS > 1 && LS * RL == NP, "radix plan");
  const int tid = threadIdx.x;
  if (tid < NG1) {
    // first pass, span 1: no twiddles; outputs to X[j R1 + t]
    if (!INV) {
#pragma unroll
      for (int t = 0; t < R1; ++t) v[t] = conjf2(v[t]);
    }
    fft_reg<R1>(v);
#pragma unroll
    for (int t = 0; t < R1; ++t) X[pidx(tid * R1 + t)] = INV ? v[t] : conjf2(v[t]);
  }
  __syncthreads();
  fft_lds_span<NP, R1, LS, INV>(X, tw);
  // last pass, span LS (= its group count): group j reads X[j + t LS] and its
  // outputs are elements j + t LS
  constexpr int GPT = (LS + 255) / 256;
#pragma unroll
  for (int g = 0; g < GPT; ++g) {
    const int j = tid + 256 * g;
    if (j < LS) {
      float2 w[RL];
#pragma unroll
      for (int t = 0; t < RL; ++t) {
        float2 x = X[pidx(j + t * LS)];
        if (t > 0) {
          const float2 f = tw(t * j);  // NP / (NS R) = 1 in the last pass
          x = cmulf(x, INV ? f : conjf2(f));
        }
        w[t] = INV ? x : conjf2(x);
      }
      fft_reg<RL>(w);
#pragma unroll
      for (int t = 0; t < RL; ++t) store(j + t * LS, INV ? w[t] : conjf2(w[t]));
    }
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
