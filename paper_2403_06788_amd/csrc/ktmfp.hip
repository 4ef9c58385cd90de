// Coarse stage of DS-KT-MFP (Alg. 4, Prop. 3, eqs. (25)-(26), P = 2) on the
// range spectrum S[m][k] of the frequency-domain mGIFT (zero-padded length NP,
// signed index k_s, eps_k = f_k / (f_c + f_k) = k_s / (R NP + k_s)).
//
//  * k_keystone: the keystone transform, band-limited interpolation of every
//    frequency's slow-time sequence at the stretched times m (1 - eps_k):
//      S_KT[m][k] = sum_{m' < M} S[m'][k] sinc(m - m' - m eps_k).
//    With m eps_k = xi + xf (xi the nearest integer, |xf| <= 1/2, from FP64)
//    and J = m - xi - m', sin(pi (J - xf)) = -(-1)^J sin(pi xf), so
//      S_KT[m][k] = -(sin(pi xf) / pi) (-1)^(m - xi)
//                     sum_m' (-1)^m' S[m'][k] / (J - xf),
//    one reciprocal and two FMAs per term in FP32; J - xf is formed from the
//    exact integer J, so the J = 0 term keeps full relative accuracy.  When
//    xf = 0 (m eps_k an integer) the sum is replaced by the exact shift
//    S[m - xi][k].  A workgroup owns KC = 8192 / M frequencies and all M
//    pulses, with (-1)^m' S staged in LDS (64 KiB).
//  * k_kt_shift: per coarse cell (q, i2c) and pulse, the folding-factor and
//    coarse-acceleration compensation H_KT,RM of eq. (26) and the IFFT over
//    range frequency:
//      E[u][m][r] = (1/NP) sum_k S_KT[m][k]
//                   exp(+j 2 pi (q m eps_k - k_s x2(m) / NP + k (n_begin + r) / NP)),
//    x2(m) = i2c m^2 / (R M^2) the coarse acceleration walk in bins.  The turn
//    count q m k_s / (R NP + k_s) is an exact integer product times a
//    correctly rounded FP64 reciprocal (error ~1e-13 turns); k_s x2 / NP is
//    split as ((k_s xi2) mod NP) / NP + k_s xf2 / NP.  The reduced turns go
//    through FP32 sincospi.
// The rows E[u] then pass through the FP32 gather with zero offsets and the
// pre-DFM phase exp(+j 2 pi i2c m^2 M / M^3) of the unit tables (the folded
// velocity q M contributes whole turns), and the fine FFT search over the M
// baseband velocities and R fine accelerations.
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

constexpr int KS_LDS = 8192;  // complex64 entries of the keystone's LDS tile

__global__ void k_kt_invd(int NP, int R, double *invd) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < NP) {
    const int ks = k < NP / 2 ? k : k - NP;
    invd[k] = 1.0 / ((double)R * (double)NP + (double)ks);
  }
}

// J = 32 outputs per thread: thread t of column kc handles pulses
// m = t + TPC j, j < 32.
template <int M>
__global__ __launch_bounds__(256) void k_keystone(const float2 *__restrict__ spec,
                                                  const double *__restrict__ invd,
                                                  int NP, float2 *__restrict__ out) {
  constexpr int KC = KS_LDS / M;
  constexpr int TPC = 256 / KC;
  constexpr int J = M / TPC;
  static_assert(J == 32 && TPC * KC == 256, "keystone tiling");
  __shared__ float2 s_S[M * KC];  // [m'][kc] = (-1)^m' S[m'][k0 + kc]
  const int tid = threadIdx.x;
  const int k0 = blockIdx.x * KC;
  for (int i = tid; i < M * KC; i += 256) {
    const int mp = i / KC, c = i % KC;
    float2 v = make_float2(0.f, 0.f);
    if (k0 + c < NP) v = spec[(int64_t)mp * NP + k0 + c];
    if (mp & 1) v = make_float2(-v.x, -v.y);
    s_S[i] = v;
  }
  const int kc = tid / TPC, t = tid % TPC;
  const int k = k0 + kc;
  const int kk = k < NP ? k : 0;
  const int ks = kk < NP / 2 ? kk : kk - NP;
  const double id = invd[kk];
  float cj[J], xf[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int m = t + TPC * j;
    const double x = (double)((int64_t)m * ks) * id;  // m eps_k
    const double r = rint(x);
    xf[j] = (float)(x - r);
    cj[j] = (float)(m - (int)r);
  }
  __syncthreads();
  float2 acc[J];
#pragma unroll
  for (int j = 0; j < J; ++j) acc[j] = make_float2(0.f, 0.f);
  for (int mp = 0; mp < M; ++mp) {
    const float2 v = s_S[mp * KC + kc];
    const float fm = (float)mp;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const float d = (cj[j] - fm) - xf[j];   // J - xf, J exact
      const float rc = __builtin_amdgcn_rcpf(d);
      acc[j].x = fmaf(v.x, rc, acc[j].x);
      acc[j].y = fmaf(v.y, rc, acc[j].y);
    }
  }
  if (k < NP) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int m = t + TPC * j;
      float2 y;
      const int src = (int)cj[j];  // m - xi
      if (xf[j] == 0.f) {
        // exact shift; s_S holds (-1)^src S[src], and (-1)^(2 src) = 1
        y = make_float2(0.f, 0.f);
        if (src >= 0 && src < M) {
          y = s_S[src * KC + kc];
          if (src & 1) y = make_float2(-y.x, -y.y);
        }
      } else {
        float sc = -sinpif(xf[j]) * 0.318309886183790672f;  // -sin(pi xf) / pi
        if (src & 1) sc = -sc;
        y = make_float2(sc * acc[j].x, sc * acc[j].y);
      }
      out[(int64_t)m * NP + k] = y;
    }
  }
}

template <int NP>
__global__ __launch_bounds__(256) void k_kt_shift(
    const float2 *__restrict__ kspec, const float2 *__restrict__ tw,
    const double *__restrict__ invd, const int64_t *cells, int64_t cc_base,
    int64_t unit0, int M, int R, int q_lo, int n_a, int ilo1, int rows, int rows_p,
    int n_begin, float2 *__restrict__ E) {
  __shared__ float2 X[lds_len<NP>()];
  __shared__ float2 t_lo[128], t_hi[NP / 128 > 1 ? NP / 128 : 1];
  const TwLds tl = load_twiddles<NP>(tw, t_lo, t_hi);
  const int tid = threadIdx.x;
  const int64_t u = blockIdx.x / M;
  const int m = (int)(blockIdx.x % M);
  const int64_t k = cell_id(cells, cc_base, unit0 + u);
  const int64_t q = q_lo + k % n_a;
  const int64_t i2c = ilo1 + (k / n_a) * R + R / 2;
  const double g = (double)(q * m);                      // q m, exact
  const int64_t RM2 = (int64_t)R * M * M;
  const int64_t num2 = i2c * m * m;
  const int64_t xi2 = floor_div(num2, RM2);
  const double xf2 = (double)(num2 - xi2 * RM2) / (double)RM2;
  // the first pass's elements straight from the spectrum (thread j < NP / R1
  // takes k = j + t NP / R1, coalesced over j); the FP64 reciprocals in
  // groups of LB, all of a group's loads issued before the first is used
  constexpr int R1 = first_radix<NP>(), NG1 = NP / R1, LB = R1 < 8 ? R1 : 8;
  const float2 *sp = kspec + (int64_t)m * NP;
  float2 v[R1];
  if (tid < NG1) {
#pragma unroll
    for (int t = 0; t < R1; ++t) v[t] = sp[tid + t * NG1];
#pragma unroll
    for (int t0 = 0; t0 < R1; t0 += LB) {
      double iv[LB];
#pragma unroll
      for (int e = 0; e < LB; ++e) iv[e] = invd[tid + (t0 + e) * NG1];
#pragma unroll
      for (int e = 0; e < LB; ++e) {
        const int kk = tid + (t0 + e) * NG1;
        const int ks = kk < NP / 2 ? kk : kk - NP;
        const int ii = (int)(((int64_t)ks * xi2) & (NP - 1));   // (k_s xi2) mod NP
        double turns = g * (double)ks * iv[e] -
                       ((double)ii + (double)ks * xf2) * (1.0 / (double)NP);
        turns -= rint(turns);
        float s, c;
        sincospif(2.0f * (float)turns, &s, &c);
        v[t0 + e] = cmulf(v[t0 + e], make_float2(c, s));
      }
    }
  }
  // outputs n_begin + r straight to the unit's row; rows from rows to rows_p
  // are zero (those past the transform's end below)
  const float inv = 1.0f / (float)NP;
  float2 *o = E + ((int64_t)u * M + m) * rows_p;
  fft_lds_io<NP, true>(v, X, tl, [&](int i, float2 y) {
    const int r = i - n_begin;
    if (r >= 0 && r < rows_p)
      o[r] = (r < rows) ? make_float2(y.x * inv, y.y * inv) : make_float2(0.f, 0.f);
  });
  for (int r = (NP - n_begin > 0 ? NP - n_begin : 0) + tid; r < rows_p; r += 256)
    o[r] = make_float2(0.f, 0.f);
}

template <int M>
hipError_t keystone_m(dsgrft_plan p, hipStream_t s) {
  constexpr int KC = KS_LDS / M;
  const int blocks = (p->fd_np + KC - 1) / KC;
  hipLaunchKernelGGL((k_keystone<M>), dim3(blocks), dim3(256), 0, s, p->fd_spec,
                     p->kt_invd, p->fd_np, p->kt_spec);
  return hipGetLastError();
}

template <int NP>
hipError_t shift_np(dsgrft_plan p, const int64_t *cells, int64_t cc_base,
                    int64_t unit0, int64_t nunits, hipStream_t s) {
  hipLaunchKernelGGL((k_kt_shift<NP>), dim3((unsigned)(nunits * p->M)), dim3(256), 0, s,
                     p->kt_spec, p->fd_tw, p->kt_invd, cells, cc_base, unit0, p->M, p->R,
                     p->kt_q_lo, p->kt_na, p->ilo[1], p->rows, p->rows_p, p->n_begin,
                     p->fd_E);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_kt_tables(dsgrft_plan p, hipStream_t s) {
  hipLaunchKernelGGL(k_kt_invd, dim3((p->fd_np + 255) / 256), dim3(256), 0, s, p->fd_np,
                     p->R, p->kt_invd);
  return hipGetLastError();
}

hipError_t launch_keystone(dsgrft_plan p, hipStream_t s) {
  switch (p->M) {
    case 64: return keystone_m<64>(p, s);
    case 128: return keystone_m<128>(p, s);
    case 256: return keystone_m<256>(p, s);
    case 512: return keystone_m<512>(p, s);
    case 1024: return keystone_m<1024>(p, s);
    case 2048: return keystone_m<2048>(p, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_kt_shift(dsgrft_plan p, const int64_t *cells, int64_t cc_base,
                           int64_t unit0, int64_t nunits, hipStream_t s) {
  switch (p->fd_np) {
    case 64: return shift_np<64>(p, cells, cc_base, unit0, nunits, s);
    case 128: return shift_np<128>(p, cells, cc_base, unit0, nunits, s);
    case 256: return shift_np<256>(p, cells, cc_base, unit0, nunits, s);
    case 512: return shift_np<512>(p, cells, cc_base, unit0, nunits, s);
    case 1024: return shift_np<1024>(p, cells, cc_base, unit0, nunits, s);
    case 2048: return shift_np<2048>(p, cells, cc_base, unit0, nunits, s);
    case 4096: return shift_np<4096>(p, cells, cc_base, unit0, nunits, s);
    case 8192: return shift_np<8192>(p, cells, cc_base, unit0, nunits, s);
    case 16384: return shift_np<16384>(p, cells, cc_base, unit0, nunits, s);
    default: return hipErrorInvalidValue;
  }
}
