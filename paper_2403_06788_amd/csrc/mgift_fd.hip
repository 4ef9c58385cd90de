// Frequency-domain mGIFT (Alg. 1, eq. (46) with H_RM of eq. (10)) on the
// range-compressed echo.
//
//  * k_range_fft: per pulse, the range spectrum of the row zero-padded to NP
//    (a power of two >= N + W, W a bound of the coarse walk in bins, so that
//    an integer walk never wraps into the window):
//      S[m][k] = sum_{n<N} s[m][n] exp(-j 2 pi k n / NP);
//  * k_fd_shift: per gathered unit and pulse, the coarse RM compensation and
//    the IFFT over range frequency,
//      E[u][m][r] = (1/NP) sum_k S[m][k] exp(+j 2 pi k_s x(m) / NP)
//                                   exp(+j 2 pi k (n_begin + r) / NP),
//    with k_s the signed frequency index (k, or k - NP from NP/2 on) and
//    x(m) = Num_c(m) / (R M^3) the coarse walk of the unit's cell in bins.
//    The phase k_s x / NP is formed as ((k_s xi) mod NP) / NP + k_s xf / NP
//    with xi = floor(x) exact and xf in [0, 1) in FP64; the second factor is
//    a product of two small tables (k_s = 64 a + c) whose phases are reduced
//    in FP64.
// The rows E[u] then go through the ordinary gathers with zero offsets, which
// apply the pre-DFM phase (eq. (47)) and write the fine search's layout.
//
// Both transforms are Stockham autosort FFTs in LDS, one workgroup of 256
// threads per row: pass with span NS and radix R reads X[j + t NP/R], scales
// by W^(t (j mod NS)), runs an R-point FFT in registers and writes
// X[(j/NS) NS R + (j mod NS) + t NS].  Every thread loads all its groups
// before the barrier and writes after it, so the pass works in place.  The
// radices are 16 with the remainder folded into the first pass (32 or 64) or
// a last pass of 4 or 8, so NP = 8192 takes three passes.  Twiddles come from
// two small LDS tables, W^i = TH[i >> 7] TL[i & 127].
#include "fft_reg.h"
#include "internal.h"

namespace {

using fftreg::cmulf;
using fftreg::fft_reg;

__device__ inline float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

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
        float2 x = X[j + t * NG];
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
      for (int t = 0; t < R; ++t) X[d + t * NS] = INV ? v[g][t] : conjf2(v[g][t]);
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

template <int NP>
__global__ __launch_bounds__(256) void k_range_fft(const float2 *__restrict__ echo,
                                                   int N, const float2 *__restrict__ tw,
                                                   float2 *__restrict__ spec) {
  __shared__ float2 X[NP];
  __shared__ float2 t_lo[128], t_hi[NP / 128 > 1 ? NP / 128 : 1];
  const TwLds tl = load_twiddles<NP>(tw, t_lo, t_hi);
  const int m = blockIdx.x;
  for (int n = threadIdx.x; n < NP; n += 256)
    X[n] = (n < N) ? echo[(int64_t)m * N + n] : make_float2(0.f, 0.f);
  __syncthreads();
  fft_lds<NP, 1, false>(X, tl);
  for (int k = threadIdx.x; k < NP; k += 256) spec[(int64_t)m * NP + k] = X[k];
}

template <int NP>
__global__ __launch_bounds__(256) void k_fd_shift(
    const float2 *__restrict__ spec, const float2 *__restrict__ tw,
    const int64_t *cells, int64_t cc_base, int64_t unit0, int M, int R3, int R,
    int P, int K0, int K1, int K2, int i0, int i1, int i2, Lat L, int rows,
    int rows_p, int n_begin, float2 *__restrict__ E) {
  __shared__ float2 X[NP];
  constexpr int A0 = (NP + 127) / 128;            // -min(a), k_s = 64 a + c
  constexpr int NA = NP / 64 > 2 ? NP / 64 : 2;
  __shared__ float2 TA[NA], TC[64];
  __shared__ float2 t_lo[128], t_hi[NP / 128 > 1 ? NP / 128 : 1];
  const TwLds tl = load_twiddles<NP>(tw, t_lo, t_hi);
  const int tid = threadIdx.x;
  const int64_t u = blockIdx.x / M;
  const int m = (int)(blockIdx.x % M);
  const int64_t cpos = (unit0 + u) / R3;
  const int64_t k = cell_id(cells, cc_base, cpos);
  const int Ks[3] = {K0, K1, K2}, il[3] = {i0, i1, i2};
  int64_t ic[3];
  coarse_centre(Ks, il, R, P, k, ic);
  const int64_t num = lat_num(L, m, ic[0], ic[1], ic[2]);
  const int64_t xi = floor_div(num, L.RM3);
  const double xf = (double)(num - xi * L.RM3) / (double)L.RM3;
  // sub-ramp factors: the turn fractions (|.| <= 1/2) are formed in FP64 and
  // their sine and cosine taken in FP32 (error ~ FP32 rounding of the result)
  for (int i = tid; i < NA + 64; i += 256) {
    const double turns = (i < NA) ? 64.0 * (double)(i - A0) * xf / NP
                                  : (double)(i - NA) * xf / NP;
    float s, c;
    sincospif(2.0f * (float)turns, &s, &c);
    if (i < NA) TA[i] = make_float2(c, s);
    else TC[i - NA] = make_float2(c, s);
  }
  __syncthreads();
  const float2 *sp = spec + (int64_t)m * NP;
  for (int kk = tid; kk < NP; kk += 256) {
    const int ks = kk < NP / 2 ? kk : kk - NP;
    const int ii = (int)(((int64_t)ks * xi) & (NP - 1));  // (k_s xi) mod NP
    const int a = ks >> 6, c = ks & 63;                    // k_s = 64 a + c
    const float2 w = cmulf(cmulf(tl(ii), TA[a + A0]), TC[c]);
    X[kk] = cmulf(sp[kk], w);
  }
  __syncthreads();
  fft_lds<NP, 1, true>(X, tl);
  const float inv = 1.0f / (float)NP;
  float2 *out = E + ((int64_t)u * M + m) * rows_p;
  for (int r = tid; r < rows_p; r += 256) {
    const float2 y = X[n_begin + r < NP ? n_begin + r : 0];
    out[r] = (r < rows) ? make_float2(y.x * inv, y.y * inv) : make_float2(0.f, 0.f);
  }
}

__global__ void k_fd_twiddles(int NP, float2 *tw) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < NP) {
    double s, c;
    sincospi(2.0 * (double)t / (double)NP, &s, &c);
    tw[t] = make_float2((float)c, (float)s);
  }
}

template <int NP>
hipError_t launch_np(dsgrft_plan p, const float2 *echo, const int64_t *cells,
                     int64_t cc_base, int64_t unit0, int64_t nunits, int R3,
                     bool spectrum, hipStream_t s) {
  if (spectrum) {
    hipLaunchKernelGGL((k_range_fft<NP>), dim3(p->M), dim3(256), 0, s, echo, p->N,
                       p->fd_tw, p->fd_spec);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_fd_shift<NP>), dim3((unsigned)(nunits * p->M)), dim3(256), 0, s,
                     p->fd_spec, p->fd_tw, cells, cc_base, unit0, p->M, R3, p->R, p->P,
                     p->K[0], p->K[1], p->K[2], p->ilo[0], p->ilo[1], p->ilo[2], p->lat,
                     p->rows, p->rows_p, p->n_begin, p->fd_E);
  return hipGetLastError();
}

hipError_t dispatch(dsgrft_plan p, const float2 *echo, const int64_t *cells,
                    int64_t cc_base, int64_t unit0, int64_t nunits, int R3,
                    bool spectrum, hipStream_t s) {
  switch (p->fd_np) {
    case 64: return launch_np<64>(p, echo, cells, cc_base, unit0, nunits, R3, spectrum, s);
    case 128: return launch_np<128>(p, echo, cells, cc_base, unit0, nunits, R3, spectrum, s);
    case 256: return launch_np<256>(p, echo, cells, cc_base, unit0, nunits, R3, spectrum, s);
    case 512: return launch_np<512>(p, echo, cells, cc_base, unit0, nunits, R3, spectrum, s);
    case 1024: return launch_np<1024>(p, echo, cells, cc_base, unit0, nunits, R3, spectrum, s);
    case 2048: return launch_np<2048>(p, echo, cells, cc_base, unit0, nunits, R3, spectrum, s);
    case 4096: return launch_np<4096>(p, echo, cells, cc_base, unit0, nunits, R3, spectrum, s);
    case 8192: return launch_np<8192>(p, echo, cells, cc_base, unit0, nunits, R3, spectrum, s);
    case 16384: return launch_np<16384>(p, echo, cells, cc_base, unit0, nunits, R3, spectrum, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_fd_twiddles(dsgrft_plan p, hipStream_t s) {
  hipLaunchKernelGGL(k_fd_twiddles, dim3((p->fd_np + 255) / 256), dim3(256), 0, s,
                     p->fd_np, p->fd_tw);
  return hipGetLastError();
}

hipError_t launch_range_fft(dsgrft_plan p, const float2 *echo, hipStream_t s) {
  return dispatch(p, echo, nullptr, 0, 0, 0, 1, true, s);
}

hipError_t launch_fd_shift(dsgrft_plan p, const int64_t *cells, int64_t cc_base,
                           int64_t unit0, int64_t nunits, int R3, hipStream_t s) {
  return dispatch(p, nullptr, cells, cc_base, unit0, nunits, R3, false, s);
}
