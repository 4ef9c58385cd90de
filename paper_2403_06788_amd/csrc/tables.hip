// Stage a0: phase and offset tables.
//
// Fine table: H_DFM(t_m; c_f) times the fine velocity term, the matching
// phase of the GFT (eq. (44), Alg. 2), for the fine cells of orders 1..min(P,2)
// (order 3 is folded into the gathered units).  Stored once per plan in every
// arithmetic form:
//   F32   [Mp][Cp] complex64
//   F16 / FBF16  MFMA A-operand fragments of v_mfma_f32_32x32x16_{f16,bf16}:
//         planes (re_hi, im_hi, re_lo, im_lo) x (Cp/32) column blocks x
//         (Mp/16) pulse blocks x 64 lanes x 8 elements, lane l holding column
//         32 b + l % 32 and pulses 16 kb + 8 (l / 32) + e.
//   F8    fragments of the scaled 8-bit MFMA (OCP e4m3), same planes, K
//         blocks of 64 pulses (layout at the conversion below).
//
// Unit tables: for each gathered unit (coarse cell, and for P = 3 one fine
// jerk offset) the range offset of the coarse walk (the mGIFT envelope
// correction, eq. (46)) and the de-ramp phasor (H_pre-DFM of eq. (47), times
// the fine jerk phase for P = 3).  All from exact integers.
#include "internal.h"

namespace {

template <typename T>
__device__ inline uint16_t bits16(T x) {
  return __builtin_bit_cast(uint16_t, x);
}

__device__ inline uint8_t to_e4m3(float x) {
  // OCP e4m3 (bias 7, max 448), round to nearest even via the hardware
  // conversion.
  int v = __builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false);
  return (uint8_t)(v & 0xff);
}

__global__ void k_fine_tables(int M, int Mp, int C, int Cp, int R, int P, Lat L,
                              float2 *F32, uint16_t *F16, uint16_t *FB16,
                              uint8_t *F8, int KB, int FB) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)Mp * Cp) return;
  int m = (int)(t / Cp), f = (int)(t % Cp);
  double c = 0.0, s = 0.0;
  if (m < M && f < C) {
    int64_t f1, f2 = 0;
    if (P >= 2) {
      f1 = f % R - R / 2;
      f2 = f / R - R / 2;
    } else {
      f1 = f - R / 2;
    }
    int64_t num = lat_num(L, m, f1, f2, 0);
    sincospi(lat_turns2(L, num), &s, &c);
  }
  F32[(int64_t)m * Cp + f] = make_float2((float)c, (float)s);
  // 16-bit fragments
  int fb = f >> 5, kb = m >> 4;
  int lane = (f & 31) + 32 * ((m & 15) >> 3), e = m & 7;
  int64_t plane = (int64_t)FB * KB * 512;
  int64_t o = ((int64_t)fb * KB + kb) * 512 + lane * 8 + e;
  float cf = (float)c, sf = (float)s;
  _Float16 ch = (_Float16)cf, sh = (_Float16)sf;
  _Float16 cl = (_Float16)(float)(c - (double)(float)ch);
  _Float16 sl = (_Float16)(float)(s - (double)(float)sh);
  F16[o] = bits16(ch);
  F16[o + plane] = bits16(sh);
  F16[o + 2 * plane] = bits16(cl);
  F16[o + 3 * plane] = bits16(sl);
  __bf16 cb = (__bf16)cf, sb = (__bf16)sf;
  __bf16 cbl = (__bf16)(float)(c - (double)(float)cb);
  __bf16 sbl = (__bf16)(float)(s - (double)(float)sb);
  FB16[o] = bits16(cb);
  FB16[o + plane] = bits16(sb);
  FB16[o + 2 * plane] = bits16(cbl);
  FB16[o + 3 * plane] = bits16(sbl);
  if (F8) {
    // fp8 fragments of v_mfma_scale_f32_32x32x64_f8f6f4 (2 KiB each): lane l
    // holds column 32 b + l % 32 and pulses 64 kb + 32 (l / 32) + e, e < 32,
    // stored as two 1 KiB halves [e / 16][lane][e % 16].  Components are
    // kept as x = fl32(256 F), hi = e4m3(x), lo = e4m3(16 (x - hi)); the MFMA
    // block scales 2^-8 and 2^-12 undo the factors.
    int kb8 = m >> 6, lane8 = (f & 31) + 32 * ((m & 63) >> 5), e8 = m & 31;
    int KB8 = KB / 4;
    int64_t plane8 = (int64_t)FB * KB8 * 2048;
    int64_t o8 = ((int64_t)fb * KB8 + kb8) * 2048 + (e8 >> 4) * 1024 + lane8 * 16 + (e8 & 15);
    float c256 = (float)(256.0 * c), s256 = (float)(256.0 * s);
    uint8_t ch8 = to_e4m3(c256), sh8 = to_e4m3(s256);
    float chf = __builtin_amdgcn_cvt_f32_fp8(ch8, 0);
    float shf = __builtin_amdgcn_cvt_f32_fp8(sh8, 0);
    F8[o8] = ch8;
    F8[o8 + plane8] = sh8;
    F8[o8 + 2 * plane8] = to_e4m3(16.0f * (c256 - chf));
    F8[o8 + 3 * plane8] = to_e4m3(16.0f * (s256 - shf));
  }
}

// Conjugate-pair table: column c of block c / 32 holds the fragments of
// fine cell cols[c] (zero where cols[c] < 0), copied from the first `planes`
// planes of F16 (fp16: re_hi, im_hi), FBF16 (bf16: also re_lo, im_lo) or F8
// (e4m3, four planes).
// HALVES 16-byte chunks per lane and fragment: 1 for the 16-bit tables, 2
// for the e4m3 one (K blocks of 64 pulses, KB of them here).
__global__ void k_sym_table(const uint4 *__restrict__ F16, const int32_t *__restrict__ cols,
                            int FB, int FBs, int KB, int planes, int halves,
                            uint4 *__restrict__ FS) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int fr = 64 * halves;
  if (t >= (int64_t)planes * FBs * KB * fr) return;
  const int lane = (int)(t & 63), h = (int)((t >> 6) % halves);
  const int64_t q = t / fr;
  const int kb = (int)(q % KB), cb = (int)((q / KB) % FBs), plane = (int)(q / ((int64_t)KB * FBs));
  const int f = cols[cb * 32 + (lane & 31)];
  FS[t] = f < 0 ? make_uint4(0u, 0u, 0u, 0u)
                : F16[(((int64_t)plane * FB + (f >> 5)) * KB + kb) * fr + h * 64 + (f & 31) +
                      32 * (lane >> 5)];
}

__global__ void k_unit_tables(const int64_t *cells, int64_t cc_base,
                              int64_t unit0, int64_t nunits, int M, int Mp,
                              int R3, int R, int P, int K0, int K1, int K2,
                              int i0, int i1, int i2, int S0, Lat L,
                              int zero_off, int32_t *off, float2 *psi) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nunits * Mp) return;
  int64_t u = t / Mp;
  int m = (int)(t % Mp);
  int32_t o = 0;
  float2 z = make_float2(0.f, 0.f);
  if (m < M) {
    int64_t ug = unit0 + u;
    int64_t cpos = ug / R3, u3 = ug % R3;
    int64_t k = cell_id(cells, cc_base, cpos);
    int Ks[3] = {K0, K1, K2}, il[3] = {i0, i1, i2};
    int64_t ic[3];
    coarse_centre(Ks, il, R, P, k, ic, S0);
    int64_t num_c = lat_num(L, m, ic[0], ic[1], ic[2]);
    o = zero_off ? 0 : lat_offset(L, num_c);
    int64_t f3 = (P == 3) ? (u3 - R / 2) : 0;
    z = lat_phasor(L, num_c + f3 * (int64_t)m * m * m);
  }
  off[t] = o;
  psi[t] = z;
}

__global__ void k_coarse_tables(int64_t cc_begin, int64_t n, int M, int stride,
                                int R, int P, int K0, int K1, int K2, int i0,
                                int i1, int i2, int S0, Lat L, int zero_off,
                                int32_t *off, float2 *psi) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * M) return;
  int64_t i = t / M;
  int64_t k = cc_begin + i;
  int m = (int)(t % M);
  int Ks[3] = {K0, K1, K2}, il[3] = {i0, i1, i2};
  int64_t ic[3];
  coarse_centre(Ks, il, R, P, k, ic, S0);
  int64_t num = lat_num(L, m, ic[0], ic[1], ic[2]);
  off[i * stride + m] = zero_off ? 0 : lat_offset(L, num);
  psi[i * stride + m] = lat_phasor(L, num);
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_fine_tables(dsgrft_plan p, hipStream_t s) {
  int64_t n = (int64_t)p->Mp * p->Cp;
  hipLaunchKernelGGL(k_fine_tables, dim3(blocks(n, 256)), dim3(256), 0, s, p->M,
                     p->Mp, p->C, p->Cp, p->R, p->P, p->lat, p->F32,
                     (uint16_t *)p->F16, (uint16_t *)p->FBF16,
                     (uint8_t *)p->F8, p->KB, p->FB);
  return hipGetLastError();
}

hipError_t launch_sym_table(dsgrft_plan p, hipStream_t s) {
  const int64_t n = (int64_t)2 * p->FBs * p->KB * 64;
  hipLaunchKernelGGL(k_sym_table, dim3(blocks(n, 256)), dim3(256), 0, s, p->F16,
                     p->sym_cols, p->FB, p->FBs, p->KB, 2, 1, p->FS16);
  hipLaunchKernelGGL(k_sym_table, dim3(blocks(2 * n, 256)), dim3(256), 0, s, p->FBF16,
                     p->sym_cols, p->FB, p->FBs, p->KB, 4, 1, p->FSB16);
  // e4m3: 4 planes x KB / 4 blocks x 128 chunks = n chunks
  if (p->FS8)
    hipLaunchKernelGGL(k_sym_table, dim3(blocks(n, 256)), dim3(256), 0, s,
                       (const uint4 *)p->F8, p->sym_cols, p->FB, p->FBs, p->KB / 4, 4, 2,
                       p->FS8);
  return hipGetLastError();
}

hipError_t launch_unit_tables(dsgrft_plan p, const int64_t *cells,
                              int64_t cc_base, int64_t unit0, int64_t nunits,
                              hipStream_t s) {
  int64_t n = nunits * p->Mp;
  hipLaunchKernelGGL(k_unit_tables, dim3(blocks(n, 256)), dim3(256), 0, s,
                     cells, cc_base, unit0, nunits, p->M, p->Mp, p->R3, p->R,
                     p->P, p->K[0], p->K[1], p->K[2], p->ilo[0], p->ilo[1],
                     p->ilo[2], p->S0, p->lat, p->fd, p->u_off, p->u_psi);
  return hipGetLastError();
}

hipError_t launch_coarse_tables(dsgrft_plan p, int64_t cc_begin, int64_t n,
                                int stride, int32_t *off, float2 *psi,
                                hipStream_t s, bool zero_off) {
  int64_t tot = n * p->M;
  hipLaunchKernelGGL(k_coarse_tables, dim3(blocks(tot, 256)), dim3(256), 0, s,
                     cc_begin, n, p->M, stride, p->R, p->P, p->K[0], p->K[1], p->K[2],
                     p->ilo[0], p->ilo[1], p->ilo[2], p->S0, p->lat, zero_off ? 1 : 0,
                     off, psi);
  return hipGetLastError();
}
