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
//    A turn count n x / NP is formed as ((n xi) mod NP) / NP + n xf / NP
//    with xi = floor(x) exact and xf in [0, 1) in FP64.  The thread that
//    loads k = j + t NP/R1 (the FFT's first pass) takes the ramp as the
//    product of exp(+j 2 pi j x / NP), its own, and exp(+j 2 pi (k_s - j) x
//    / NP), one of R1 per workgroup.
// The rows E[u] then go through the ordinary gathers with zero offsets, which
// apply the pre-DFM phase (eq. (47)) and write the fine search's layout.
//
// Both transforms are the LDS Stockham FFTs of fft_lds.h, one workgroup of
// 256 threads per row.
#include "fft_lds.h"
#include "internal.h"

namespace {

using fftreg::cmulf;
using fftlds::TwLds;
using fftlds::fft_lds;
using fftlds::fft_lds_io;
using fftlds::first_radix;
using fftlds::load_twiddles;
using fftlds::lds_len;
using fftlds::pidx;

template <int NP>
__global__ __launch_bounds__(256) void k_range_fft(const float2 *__restrict__ echo,
                                                   int N, const float2 *__restrict__ tw,
                                                   float2 *__restrict__ spec) {
  __shared__ float2 X[lds_len<NP>()];
  __shared__ float2 t_lo[128], t_hi[NP / 128 > 1 ? NP / 128 : 1];
  const TwLds tl = load_twiddles<NP>(tw, t_lo, t_hi);
  const int m = blockIdx.x;
  // loads in groups of LB per thread, all issued before the first is used
  constexpr int EPT = (NP + 255) / 256, LB = EPT < 16 ? EPT : 16;
  for (int e0 = 0; e0 < EPT; e0 += LB) {
    float2 sv[LB];
#pragma unroll
    for (int e = 0; e < LB; ++e) {
      const int n = threadIdx.x + 256 * (e0 + e);
      sv[e] = (n < N && n < NP) ? echo[(int64_t)m * N + n] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int e = 0; e < LB; ++e) {
      const int n = threadIdx.x + 256 * (e0 + e);
      if (n < NP) X[pidx(n)] = sv[e];
    }
  }
  __syncthreads();
  fft_lds<NP, 1, false>(X, tl);
  for (int k = threadIdx.x; k < NP; k += 256) spec[(int64_t)m * NP + k] = X[pidx(k)];
}

template <int NP>
__global__ __launch_bounds__(256) void k_fd_shift(
    const float2 *__restrict__ spec, const float2 *__restrict__ tw,
    const int64_t *cells, int64_t cc_base, int64_t unit0, int M, int R3, int R,
    int P, int K0, int K1, int K2, int i0, int i1, int i2, Lat L, int rows,
    int rows_p, int n_begin, float2 *__restrict__ E) {
  constexpr int R1 = first_radix<NP>(), NG1 = NP / R1;
  __shared__ float2 X[lds_len<NP>()];
  __shared__ float2 TP[R1];
  __shared__ float2 t_lo[128], t_hi[NP / 128 > 1 ? NP / 128 : 1];
  const TwLds tl = load_twiddles<NP>(tw, t_lo, t_hi);
  const int tid = threadIdx.x;
  const int64_t u = blockIdx.x / M;
  const int m = (int)(blockIdx.x % M);
  const int64_t cpos = (unit0 + u) / R3;
  const int64_t k = cell_id(cells, cc_base, cpos);
  const int Ks[3] = {K0, K1, K2}, il[3] = {i0, i1, i2};
  int64_t ic[3];
  coarse_centre(Ks, il, R, P, k, ic, R);
  const int64_t num = lat_num(L, m, ic[0], ic[1], ic[2]);
  const int64_t xi = floor_div(num, L.RM3);
  const double xf = (double)(num - xi * L.RM3) / (double)L.RM3;
  // exp(+j 2 pi n x / NP): the turns reduced in FP64 (|.| <= 1/2), their
  // sine and cosine in FP32 (error ~ FP32 rounding of the result)
  auto ramp = [&](int64_t n) {
    const int64_t ii = (n * xi) & (NP - 1);  // (n xi) mod NP, n xi exact
    double turns = ((double)ii + (double)n * xf) / (double)NP;
    turns -= rint(turns);
    float s, c;
    sincospif(2.0f * (float)turns, &s, &c);
    return make_float2(c, s);
  };
  // k = j + t NG1 has k_s - j = t NG1, less NP from t = R1 / 2 on
  if (tid < R1) TP[tid] = ramp((int64_t)tid * NG1 - (tid >= R1 / 2 ? NP : 0));
  const float2 rj = ramp(tid);
  __syncthreads();
  // the first pass's elements straight from the spectrum (thread j < NP / R1
  // takes k = j + t NP / R1, coalesced over j), all loads issued before the
  // first is used
  const float2 *sp = spec + (int64_t)m * NP;
  float2 v[R1];
  if (tid < NG1) {
#pragma unroll
    for (int t = 0; t < R1; ++t) v[t] = sp[tid + t * NG1];
#pragma unroll
    for (int t = 0; t < R1; ++t) v[t] = cmulf(v[t], cmulf(rj, TP[t]));
  }
  // outputs n_begin + r straight to the unit's row; rows from rows to rows_p
  // are zero (those past the transform's end below)
  const float inv = 1.0f / (float)NP;
  float2 *out = E + ((int64_t)u * M + m) * rows_p;
  fft_lds_io<NP, true>(v, X, tl, [&](int i, float2 y) {
    const int r = i - n_begin;
    if (r >= 0 && r < rows_p)
      out[r] = (r < rows) ? make_float2(y.x * inv, y.y * inv) : make_float2(0.f, 0.f);
  });
  for (int r = (NP - n_begin > 0 ? NP - n_begin : 0) + tid; r < rows_p; r += 256)
    out[r] = make_float2(0.f, 0.f);
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
