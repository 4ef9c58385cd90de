// Stages a1 + a2: mGIFT in the time domain (eq. (46), Alg. 1).
//
// For every gathered unit u and range row r the slow-time sequence
//   G[u][m][r] = S(m, n_begin + r + off[u][m]) * psi[u][m]
// (S = 0 outside [0, N)) is read along the coarse walk and de-ramped by the
// coarse pre-DFM phase.  Reads of the echo are coalesced along the range
// axis (a unit's walk is the same shift for every row of one pulse).
//
// Two output layouts:
//  * FP32 plain form: complex64 [u][Mp][rows_p], row-contiguous.
//  * MFMA forms: B-operand fragments of v_mfma_f32_32x32x16_{f16,bf16}:
//    planes (re_hi, im_hi[, re_lo, im_lo]) x (rows_p/32) row blocks x
//    (Mp/16) pulse blocks x 64 lanes x 8 elements; lane l holds row
//    32 nb + l % 32 and pulses 16 kb + 8 (l / 32) + e.  One wave writes one
//    1 KiB fragment per plane, contiguously.
#include "internal.h"

namespace {

__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline float2 sample(const float2 *__restrict__ echo, int N, int m,
                                int idx) {
  return (idx >= 0 && idx < N) ? echo[(int64_t)m * N + idx] : make_float2(0.f, 0.f);
}

__global__ void k_gather_f32(const float2 *__restrict__ echo,
                             const int32_t *__restrict__ off,
                             const float2 *__restrict__ psi, int M, int N,
                             int Mp, int rows, int rows_p, int n_begin,
                             int64_t nunits, float2 *__restrict__ G) {
  const int rb = (rows_p + 255) / 256;
  const int64_t um = (int64_t)blockIdx.x / rb;  // u * Mp + m
  const int r = (int)(blockIdx.x % rb) * 256 + threadIdx.x;
  if (r >= rows_p) return;
  int m = (int)(um % Mp);
  float2 v = make_float2(0.f, 0.f);
  if (m < M && r < rows) {
    int idx = n_begin + r + off[um];
    v = cmul(sample(echo, N, m, idx), psi[um]);
  }
  G[um * rows_p + r] = v;
}

__global__ void k_mgift_out(const float2 *__restrict__ echo,
                            const int32_t *__restrict__ off,
                            const float2 *__restrict__ psi, int M, int N, int Mp,
                            int rows, int n_begin, float2 *__restrict__ out) {
  const int rb = (rows + 255) / 256;
  const int64_t um0 = (int64_t)blockIdx.x / rb;  // u * M + m
  const int r = (int)(blockIdx.x % rb) * 256 + threadIdx.x;
  const int64_t u = um0 / M;
  const int m = (int)(um0 % M);
  if (r >= rows) return;
  int64_t um = u * Mp + m;
  int idx = n_begin + r + off[um];
  out[((int64_t)u * M + m) * rows + r] = cmul(sample(echo, N, m, idx), psi[um]);
}

template <typename T>
__device__ inline uint16_t b16(T x) {
  return __builtin_bit_cast(uint16_t, x);
}

template <typename T, int NP>
__global__ __launch_bounds__(256) void k_gather_lp(
    const float2 *__restrict__ echo, const int32_t *__restrict__ off,
    const float2 *__restrict__ psi, int M, int N, int Mp, int rows, int n_begin,
    int NB, int KB, int64_t nunits, uint4 *__restrict__ G) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= nunits * NB * KB) return;
  const int kb = (int)(w % KB);
  const int nb = (int)((w / KB) % NB);
  const int64_t u = w / ((int64_t)KB * NB);
  const int r = nb * 32 + (lane & 31);
  const int m0 = kb * 16 + 8 * (lane >> 5);
  uint16_t re_h[8], im_h[8], re_l[8], im_l[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    int m = m0 + e;
    float2 v = make_float2(0.f, 0.f);
    if (m < M && r < rows) {
      int64_t um = u * Mp + m;
      v = cmul(sample(echo, N, m, n_begin + r + off[um]), psi[um]);
    }
    T hr = (T)v.x, hi = (T)v.y;
    re_h[e] = b16(hr);
    im_h[e] = b16(hi);
    if (NP == 4) {
      re_l[e] = b16((T)(v.x - (float)hr));
      im_l[e] = b16((T)(v.y - (float)hi));
    }
  }
  auto pack = [](const uint16_t *h) {
    return make_uint4(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16),
                      h[4] | ((uint32_t)h[5] << 16), h[6] | ((uint32_t)h[7] << 16));
  };
  const int64_t plane = (int64_t)NB * KB * 64;
  const int64_t o = ((u * NP) * NB + nb) * (int64_t)KB * 64 + (int64_t)kb * 64 + lane;
  G[o] = pack(re_h);
  G[o + plane] = pack(im_h);
  if (NP == 4) {
    G[o + 2 * plane] = pack(re_l);
    G[o + 3 * plane] = pack(im_l);
  }
}

}  // namespace

hipError_t launch_gather_f32(dsgrft_plan p, const float2 *echo, int64_t nunits,
                             hipStream_t s) {
  dim3 grid((unsigned)(((p->rows_p + 255) / 256) * nunits * p->Mp));
  hipLaunchKernelGGL(k_gather_f32, grid, dim3(256), 0, s, echo, p->u_off, p->u_psi,
                     p->M, p->N, p->Mp, p->rows, p->rows_p, p->n_begin, nunits,
                     (float2 *)p->G);
  return hipGetLastError();
}

hipError_t launch_mgift_out(dsgrft_plan p, const float2 *echo, int64_t nunits,
                            float2 *out, hipStream_t s) {
  dim3 grid((unsigned)(((p->rows + 255) / 256) * nunits * p->M));
  hipLaunchKernelGGL(k_mgift_out, grid, dim3(256), 0, s, echo, p->u_off, p->u_psi,
                     p->M, p->N, p->Mp, p->rows, p->n_begin, out);
  return hipGetLastError();
}

hipError_t launch_gather_lp(dsgrft_plan p, dsgrft_form form, int split,
                            const float2 *echo, int64_t nunits, hipStream_t s) {
  int64_t waves = nunits * p->NB * p->KB;
  dim3 grid((unsigned)((waves + 3) / 4));
  uint4 *G = (uint4 *)p->G;
  if (form == DSGRFT_FORM_F16) {
    if (split == 1)
      hipLaunchKernelGGL((k_gather_lp<_Float16, 2>), grid, dim3(256), 0, s, echo,
                         p->u_off, p->u_psi, p->M, p->N, p->Mp, p->rows,
                         p->n_begin, p->NB, p->KB, nunits, G);
    else
      hipLaunchKernelGGL((k_gather_lp<_Float16, 4>), grid, dim3(256), 0, s, echo,
                         p->u_off, p->u_psi, p->M, p->N, p->Mp, p->rows,
                         p->n_begin, p->NB, p->KB, nunits, G);
  } else if (form == DSGRFT_FORM_BF16) {
    if (split == 1)
      hipLaunchKernelGGL((k_gather_lp<__bf16, 2>), grid, dim3(256), 0, s, echo,
                         p->u_off, p->u_psi, p->M, p->N, p->Mp, p->rows,
                         p->n_begin, p->NB, p->KB, nunits, G);
    else
      hipLaunchKernelGGL((k_gather_lp<__bf16, 4>), grid, dim3(256), 0, s, echo,
                         p->u_off, p->u_psi, p->M, p->N, p->Mp, p->rows,
                         p->n_begin, p->NB, p->KB, nunits, G);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
