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
//    32 nb + l % 32 and pulses 16 kb + 8 (l / 32) + e.  A wave writes whole
//    1 KiB fragments per plane, contiguously.
//    The fp16 forms store G 2^sh with one shift per echo: with mx the
//    echo's largest |Re| or |Im| component and 2^(e-1) <= mx < 2^e,
//    sh = 10 - e (0 for an all-zero echo, clamped to [-100, 100]), so the
//    largest component sits in [2^9, 2^10) whatever the echo's scale: far
//    from fp16's overflow (65504) even after the de-ramp rotation, the
//    three-product form's operand sums and the frequency-domain shift's
//    interpolation overshoot, and 2^24 above its subnormal range.  The fine
//    search scales the power back by 2^(-2 sh) (exact).
//  * 8-bit form: B-operand fragments of v_mfma_scale_f32_32x32x64_f8f6f4
//    (OCP e4m3), K blocks of 64 pulses, 2 KiB each as two halves
//    [e / 16][lane][e % 16], lane l holding row 32 nb + l % 32 and pulses
//    64 kb + 32 (l / 32) + e.  Every (unit, row) has its own power-of-two
//    scale: with mx the largest |Re S| or |Im S| over the row's walk and
//    mx = f 2^e (f in [0.5, 1)), the row is stored as x = G 2^(8 - e),
//    hi = e4m3(x), lo = e4m3(16 (x - hi)), and the E8M0 block-scale code
//    119 + e (2^(e - 8)) is written per row for the MFMA.  |x| < 256 sqrt 2
//    stays inside the e4m3 range (448).
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
                             int64_t estride, int64_t nunits,
                             float2 *__restrict__ G) {
  const int rb = (rows_p + 255) / 256;
  const int64_t um = (int64_t)blockIdx.x / rb;  // u * Mp + m
  const int r = (int)(blockIdx.x % rb) * 256 + threadIdx.x;
  if (r >= rows_p) return;
  int m = (int)(um % Mp);
  float2 v = make_float2(0.f, 0.f);
  if (m < M && r < rows) {
    int idx = n_begin + r + off[um];
    v = cmul(sample(echo + (um / Mp) * estride, N, m, idx), psi[um]);
  }
  G[um * rows_p + r] = v;
}

__global__ void k_mgift_out(const float2 *__restrict__ echo,
                            const int32_t *__restrict__ off,
                            const float2 *__restrict__ psi, int M, int N, int Mp,
                            int rows, int n_begin, int64_t estride,
                            float2 *__restrict__ out) {
  const int rb = (rows + 255) / 256;
  const int64_t um0 = (int64_t)blockIdx.x / rb;  // u * M + m
  const int r = (int)(blockIdx.x % rb) * 256 + threadIdx.x;
  const int64_t u = um0 / M;
  const int m = (int)(um0 % M);
  if (r >= rows) return;
  int64_t um = u * Mp + m;
  int idx = n_begin + r + off[um];
  out[((int64_t)u * M + m) * rows + r] = cmul(sample(echo + u * estride, N, m, idx), psi[um]);
}

template <typename T>
__device__ inline uint16_t b16(T x) {
  return __builtin_bit_cast(uint16_t, x);
}

// Echo scale of the fp16 forms: sh[0] = bits of the largest |Re|/|Im|
// component (non-negative floats order as their bit patterns), sh[1] =
// 10 - e with 2^(e-1) <= max < 2^e.
__global__ void k_shift_zero(int32_t *__restrict__ sh) {
  if (threadIdx.x == 0 && blockIdx.x == 0) sh[0] = 0;
}

__global__ __launch_bounds__(256) void k_echo_maxabs(const float2 *__restrict__ e, int64_t n,
                                                     int32_t *__restrict__ sh) {
  float mx = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const float2 v = e[i];
    mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  if ((threadIdx.x & 63) == 0) atomicMax((unsigned *)sh, __float_as_uint(mx));
}

__global__ void k_shift_final(int32_t *__restrict__ sh) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const float mx = __uint_as_float((unsigned)sh[0]);
  int e = 0;
  if (mx > 0.f) (void)frexpf(mx, &e);
  const int s = 10 - e;
  sh[1] = s < -100 ? -100 : (s > 100 ? 100 : s);
}

// One workgroup per (unit, row block of 32 rows, 4 KPW pulse blocks): the
// offsets and de-ramp phasors of its 64 KPW pulses are staged in LDS, then
// wave w writes the fragments of pulse blocks kb0 + w KPW .. + KPW - 1, so
// each lane has 8 KPW independent echo loads in flight.
constexpr int KPW = 4;

template <typename T, int NP>
__global__ __launch_bounds__(256) void k_gather_lp(
    const float2 *__restrict__ echo, const int32_t *__restrict__ off,
    const float2 *__restrict__ psi, int M, int N, int Mp, int rows, int n_begin,
    int64_t estride, int NB, int KB, int64_t nunits, const int32_t *__restrict__ shift,
    uint4 *__restrict__ G) {
  constexpr int PW = 4 * KPW * 16;  // pulses per workgroup
  __shared__ int32_t s_off[PW];
  __shared__ float2 s_psi[PW];
  const int KG = (KB + 4 * KPW - 1) / (4 * KPW);
  const int kg = (int)(blockIdx.x % KG);
  const int nb = (int)((blockIdx.x / KG) % NB);
  const int64_t u = blockIdx.x / ((int64_t)KG * NB);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mw0 = kg * PW;
  {
    const int m = mw0 + tid;
    s_off[tid] = (m < Mp) ? off[u * Mp + m] : 0;
    s_psi[tid] = (m < Mp) ? psi[u * Mp + m] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  echo += u * estride;
  const int r = nb * 32 + (lane & 31);
  const int64_t plane = (int64_t)NB * KB * 64;
  const float sc = shift != nullptr ? ldexpf(1.0f, shift[1]) : 1.0f;
  auto pack = [](const uint16_t *h) {
    return make_uint4(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16),
                      h[4] | ((uint32_t)h[5] << 16), h[6] | ((uint32_t)h[7] << 16));
  };
#pragma unroll
  for (int i = 0; i < KPW; ++i) {
    const int kb = kg * 4 * KPW + wave * KPW + i;
    const int ml0 = (wave * KPW + i) * 16 + 8 * (lane >> 5);  // local pulse
    uint16_t re_h[8], im_h[8], re_l[8], im_l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int ml = ml0 + e, m = mw0 + ml;
      float2 v = make_float2(0.f, 0.f);
      if (kb < KB && m < M && r < rows)
        v = cmul(sample(echo, N, m, n_begin + r + s_off[ml]), s_psi[ml]);
      v.x *= sc;
      v.y *= sc;
      T hr = (T)v.x, hi = (T)v.y;
      re_h[e] = b16(hr);
      im_h[e] = b16(hi);
      if (NP == 4) {
        re_l[e] = b16((T)(v.x - (float)hr));
        im_l[e] = b16((T)(v.y - (float)hi));
      }
    }
    if (kb < KB) {
      const int64_t o = ((u * NP) * NB + nb) * (int64_t)KB * 64 + (int64_t)kb * 64 + lane;
      G[o] = pack(re_h);
      G[o + plane] = pack(im_h);
      if (NP == 4) {
        G[o + 2 * plane] = pack(re_l);
        G[o + 3 * plane] = pack(im_l);
      }
    }
  }
}

__device__ inline uint32_t pack_e4m3(const float (&x)[4]) {
  int v = __builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[1], 0, false);
  v = __builtin_amdgcn_cvt_pk_fp8_f32(x[2], x[3], v, true);
  return (uint32_t)v;
}

// 16 (x - e4m3(x)) for the four bytes of a packed word.
__device__ inline void residual16(const float (&x)[4], uint32_t h, float (&r)[4]) {
  r[0] = 16.0f * (x[0] - __builtin_amdgcn_cvt_f32_fp8((int)h, 0));
  r[1] = 16.0f * (x[1] - __builtin_amdgcn_cvt_f32_fp8((int)h, 1));
  r[2] = 16.0f * (x[2] - __builtin_amdgcn_cvt_f32_fp8((int)h, 2));
  r[3] = 16.0f * (x[3] - __builtin_amdgcn_cvt_f32_fp8((int)h, 3));
}

// One workgroup per (unit, block of 32 rows): pass 1 finds each row's
// largest component over all pulses, pass 2 writes the row block's
// fragments (wave w: pulse blocks w, w + 4, ...).  When they fit (STAGED),
// the unit's offsets and de-ramp phasors are staged in LDS once; the second
// pass re-reads the walk, which the first pass has just brought into the
// caches.
template <int NP, bool STAGED>
__global__ __launch_bounds__(256) void k_gather_f8(
    const float2 *__restrict__ echo, const int32_t *__restrict__ off,
    const float2 *__restrict__ psi, int M, int N, int Mp, int rows, int rows_p,
    int n_begin, int64_t estride, int NB, int KB8, uint4 *__restrict__ G,
    int32_t *__restrict__ scale) {
  extern __shared__ char smem[];
  float2 *s_psi = (float2 *)smem;              // [Mp]
  int32_t *s_off = (int32_t *)(s_psi + Mp);     // [Mp]
  __shared__ float red[8][32];
  __shared__ float mul[32];
  const int nb = (int)(blockIdx.x % NB);
  const int64_t u = blockIdx.x / NB;
  const int t = threadIdx.x;
  echo += u * estride;
  const int32_t *uo = off + u * Mp;
  const float2 *up = psi + u * Mp;
  if (STAGED) {
    for (int m = t; m < Mp; m += 256) {
      s_off[m] = uo[m];
      s_psi[m] = up[m];
    }
    __syncthreads();
    uo = s_off;
    up = s_psi;
  }
  {
    const int r = nb * 32 + (t & 31), g = t >> 5;
    const int base = n_begin + r;
    float mx0 = 0.f, mx1 = 0.f, mx2 = 0.f, mx3 = 0.f;
    if (r < rows) {
      int m = g;
      for (; m + 24 < M; m += 32) {
        const float2 v0 = sample(echo, N, m, base + uo[m]);
        const float2 v1 = sample(echo, N, m + 8, base + uo[m + 8]);
        const float2 v2 = sample(echo, N, m + 16, base + uo[m + 16]);
        const float2 v3 = sample(echo, N, m + 24, base + uo[m + 24]);
        mx0 = fmaxf(mx0, fmaxf(fabsf(v0.x), fabsf(v0.y)));
        mx1 = fmaxf(mx1, fmaxf(fabsf(v1.x), fabsf(v1.y)));
        mx2 = fmaxf(mx2, fmaxf(fabsf(v2.x), fabsf(v2.y)));
        mx3 = fmaxf(mx3, fmaxf(fabsf(v3.x), fabsf(v3.y)));
      }
      for (; m < M; m += 8) {
        const float2 v = sample(echo, N, m, base + uo[m]);
        mx0 = fmaxf(mx0, fmaxf(fabsf(v.x), fabsf(v.y)));
      }
    }
    red[g][t & 31] = fmaxf(fmaxf(mx0, mx1), fmaxf(mx2, mx3));
  }
  __syncthreads();
  if (t < 32) {
    float mx = red[0][t];
#pragma unroll
    for (int g = 1; g < 8; ++g) mx = fmaxf(mx, red[g][t]);
    int e = 0;
    if (mx > 0.f) (void)frexpf(mx, &e);
    e = e < -100 ? -100 : (e > 100 ? 100 : e);
    mul[t] = ldexpf(1.0f, 8 - e);
    scale[u * rows_p + nb * 32 + t] = 119 + e;
  }
  __syncthreads();

  const int lane = t & 63, w = t >> 6;
  const int r = nb * 32 + (lane & 31);
  const float sm = mul[lane & 31];
  const int64_t plane = (int64_t)NB * KB8 * 128;  // uint4 per plane
  for (int kb = w; kb < KB8; kb += 4) {
    const int m0 = kb * 64 + 32 * (lane >> 5);
    uint32_t rh[8], ih[8], rl[8], il[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      float xr[4], xi[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + 4 * d + q;
        float2 v = make_float2(0.f, 0.f);
        if (m < M && r < rows)
          v = cmul(sample(echo, N, m, n_begin + r + uo[m]), up[m]);
        xr[q] = v.x * sm;
        xi[q] = v.y * sm;
      }
      rh[d] = pack_e4m3(xr);
      ih[d] = pack_e4m3(xi);
      if (NP == 4) {
        float lr[4], li[4];
        residual16(xr, rh[d], lr);
        residual16(xi, ih[d], li);
        rl[d] = pack_e4m3(lr);
        il[d] = pack_e4m3(li);
      }
    }
    const int64_t o = (((u * NP) * NB + nb) * (int64_t)KB8 + kb) * 128 + lane;
    G[o] = make_uint4(rh[0], rh[1], rh[2], rh[3]);
    G[o + 64] = make_uint4(rh[4], rh[5], rh[6], rh[7]);
    G[o + plane] = make_uint4(ih[0], ih[1], ih[2], ih[3]);
    G[o + plane + 64] = make_uint4(ih[4], ih[5], ih[6], ih[7]);
    if (NP == 4) {
      G[o + 2 * plane] = make_uint4(rl[0], rl[1], rl[2], rl[3]);
      G[o + 2 * plane + 64] = make_uint4(rl[4], rl[5], rl[6], rl[7]);
      G[o + 3 * plane] = make_uint4(il[0], il[1], il[2], il[3]);
      G[o + 3 * plane + 64] = make_uint4(il[4], il[5], il[6], il[7]);
    }
  }
}

}  // namespace

GatherSrc gather_src(dsgrft_plan p, const float2 *echo) {
  if (p->fd) return GatherSrc{p->fd_E, p->rows_p, 0, (int64_t)p->M * p->rows_p};
  return GatherSrc{echo, p->N, p->n_begin, 0};
}

hipError_t launch_gather_f32(dsgrft_plan p, GatherSrc src, int64_t nunits,
                             hipStream_t s) {
  dim3 grid((unsigned)(((p->rows_p + 255) / 256) * nunits * p->Mp));
  hipLaunchKernelGGL(k_gather_f32, grid, dim3(256), 0, s, src.echo, p->u_off, p->u_psi,
                     p->M, src.N, p->Mp, p->rows, p->rows_p, src.n_begin,
                     src.unit_stride, nunits, (float2 *)p->G);
  return hipGetLastError();
}

hipError_t launch_mgift_out(dsgrft_plan p, GatherSrc src, int64_t nunits,
                            float2 *out, hipStream_t s) {
  dim3 grid((unsigned)(((p->rows + 255) / 256) * nunits * p->M));
  hipLaunchKernelGGL(k_mgift_out, grid, dim3(256), 0, s, src.echo, p->u_off, p->u_psi,
                     p->M, src.N, p->Mp, p->rows, src.n_begin, src.unit_stride, out);
  return hipGetLastError();
}

hipError_t launch_echo_shift(dsgrft_plan p, const float2 *echo, hipStream_t s) {
  const int64_t n = (int64_t)p->M * p->N;
  const int64_t nb = (n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048;
  hipLaunchKernelGGL(k_shift_zero, dim3(1), dim3(64), 0, s, p->g_shift);
  hipLaunchKernelGGL(k_echo_maxabs, dim3((unsigned)nb), dim3(256), 0, s, echo, n, p->g_shift);
  hipLaunchKernelGGL(k_shift_final, dim3(1), dim3(64), 0, s, p->g_shift);
  return hipGetLastError();
}

hipError_t launch_gather_lp(dsgrft_plan p, dsgrft_form form, int split,
                            GatherSrc src, int64_t nunits, hipStream_t s) {
  // G's lo planes enter from split 3 on (split 2 adds the fine table's lo)
  // and in BF16_GLO and BF16_SYM
  const bool lo = split >= 3 || form == DSGRFT_FORM_BF16_GLO || form == DSGRFT_FORM_BF16_SYM;
  uint4 *G = (uint4 *)p->G;
  if (form == DSGRFT_FORM_FP8 || form == DSGRFT_FORM_FP8_SYM) {
    dim3 grid((unsigned)(nunits * p->NB));
    const size_t lds = (size_t)p->Mp * (sizeof(float2) + sizeof(int32_t));
    const bool staged = lds <= 48 * 1024;
#define DS_GATHER_F8(NP, ST)                                                          \
  hipLaunchKernelGGL((k_gather_f8<NP, ST>), grid, dim3(256), ST ? lds : 0, s, src.echo, \
                     p->u_off, p->u_psi, p->M, src.N, p->Mp, p->rows, p->rows_p,       \
                     src.n_begin, src.unit_stride, p->NB, p->KB / 4, G, p->g_scale)
    if (lo) {
      if (staged) DS_GATHER_F8(4, true); else DS_GATHER_F8(4, false);
    } else {
      if (staged) DS_GATHER_F8(2, true); else DS_GATHER_F8(2, false);
    }
#undef DS_GATHER_F8
    return hipGetLastError();
  }
  const int64_t kg = (p->KB + 4 * KPW - 1) / (4 * KPW);
  dim3 grid((unsigned)(nunits * p->NB * kg));
#define DS_GATHER_LP(T, NP, SH)                                                       \
  hipLaunchKernelGGL((k_gather_lp<T, NP>), grid, dim3(256), 0, s, src.echo, p->u_off,   \
                     p->u_psi, p->M, src.N, p->Mp, p->rows, src.n_begin,                \
                     src.unit_stride, p->NB, p->KB, nunits, SH, G)
  if (fp16_form(form)) {
    if (!lo) DS_GATHER_LP(_Float16, 2, p->g_shift); else DS_GATHER_LP(_Float16, 4, p->g_shift);
  } else if (form == DSGRFT_FORM_BF16 || form == DSGRFT_FORM_BF16_GLO ||
             form == DSGRFT_FORM_BF16_SYM) {
    if (!lo) DS_GATHER_LP(__bf16, 2, nullptr); else DS_GATHER_LP(__bf16, 4, nullptr);
  } else {
    return hipErrorInvalidValue;
  }
#undef DS_GATHER_LP
  return hipGetLastError();
}
