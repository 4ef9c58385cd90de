// Plain FP32 form of the fine search (stages a3 + a4 on the vector ALUs):
// the same Y[u][f][n] = sum_m G[u][m][n] F[m][f] as the MFMA form, with
// complex64 operands and FP32 fused multiply-adds.  It is the speed baseline
// of the MFMA forms and shares their epilogue semantics (largest power per
// (cell, row), smaller fine index on equal power).
//
// Tiling: 64 range rows x 128 fine cells per 256-thread workgroup, 16 pulses
// per LDS stage (double-buffered), 4 rows x 8 fine cells of complex
// accumulators per thread.  A thread's fine cells are strided by 16 so that
// the LDS reads of a 16-lane group are consecutive 8-byte words.
#include "internal.h"

namespace {

constexpr int TN = 64, TF = 128, KT = 16;

__device__ inline unsigned long long umax64(unsigned long long a,
                                            unsigned long long b) {
  return a > b ? a : b;
}

__device__ inline unsigned long long shfl_xor64(unsigned long long v, int m) {
  unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
  lo = __shfl_xor(lo, m);
  hi = __shfl_xor(hi, m);
  return ((unsigned long long)hi << 32) | lo;
}

__global__ __launch_bounds__(256) void k_fine_f32(
    const float2 *__restrict__ G, const float2 *__restrict__ F,
    unsigned long long *__restrict__ packed, float *__restrict__ full, int Mp,
    int rows_p, int Cp, int64_t nunits, int64_t unit0, int R3, int C, int rows) {
  __shared__ float4 sG[2][KT * TN / 2];
  __shared__ float4 sF[2][KT * TF / 2];
  const int NTt = rows_p / TN, FTt = Cp / TF;
  const int64_t bid = blockIdx.x;
  const int ft = (int)(bid % FTt);
  const int nt = (int)((bid / FTt) % NTt);
  const int64_t u = bid / ((int64_t)FTt * NTt);
  const int tid = threadIdx.x, tn = tid >> 4, tf = tid & 15;
  const int n0 = nt * TN, f0 = ft * TF;

  const float4 *Gq = (const float4 *)(G + (u * Mp) * rows_p + n0);
  const float4 *Fq = (const float4 *)(F + f0);
  const int gstride = rows_p / 2, fstride = Cp / 2;  // float4 per pulse row

  float2 acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[i][c] = make_float2(0.f, 0.f);

  const int nk = Mp / KT;
  {
    float4 rg[2], rf[4];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int q = tid + 256 * j;
      rg[j] = Gq[(int64_t)(q / 32) * gstride + (q % 32)];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = tid + 256 * j;
      rf[j] = Fq[(int64_t)(q / 64) * fstride + (q % 64)];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) sG[0][tid + 256 * j] = rg[j];
#pragma unroll
    for (int j = 0; j < 4; ++j) sF[0][tid + 256 * j] = rf[j];
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    // prefetch the next stage (the last iteration re-reads its own; that copy
    // lands in the idle buffer and is never read)
    const int k0 = ((kt + 1 < nk) ? kt + 1 : kt) * KT;
    float4 rg[2], rf[4];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int q = tid + 256 * j;
      rg[j] = Gq[(int64_t)(k0 + q / 32) * gstride + (q % 32)];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = tid + 256 * j;
      rf[j] = Fq[(int64_t)(k0 + q / 64) * fstride + (q % 64)];
    }
    const float2 *g2 = (const float2 *)sG[cur];
    const float2 *f2 = (const float2 *)sF[cur];
#pragma unroll 4
    for (int m = 0; m < KT; ++m) {
      float2 g[4], f[8];
#pragma unroll
      for (int i = 0; i < 4; ++i) g[i] = g2[m * TN + tn * 4 + i];
#pragma unroll
      for (int c = 0; c < 8; ++c) f[c] = f2[m * TF + tf + 16 * c];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          acc[i][c].x = fmaf(g[i].x, f[c].x, acc[i][c].x);
          acc[i][c].x = fmaf(-g[i].y, f[c].y, acc[i][c].x);
          acc[i][c].y = fmaf(g[i].x, f[c].y, acc[i][c].y);
          acc[i][c].y = fmaf(g[i].y, f[c].x, acc[i][c].y);
        }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) sG[cur ^ 1][tid + 256 * j] = rg[j];
#pragma unroll
    for (int j = 0; j < 4; ++j) sF[cur ^ 1][tid + 256 * j] = rf[j];
    __syncthreads();
  }

  const int64_t ug = unit0 + u;
  const int64_t cpos = ug / R3;
  const unsigned fbase = (unsigned)((ug % R3) * C);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int n = n0 + tn * 4 + i;
    unsigned long long best = 0ull;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int f = f0 + tf + 16 * c;
      const float pw = acc[i][c].x * acc[i][c].x + acc[i][c].y * acc[i][c].y;
      if (f < C) {
        const unsigned ff = fbase + (unsigned)f;
        best = umax64(best, ((unsigned long long)__float_as_uint(pw) << 32) |
                                (0xffffffffu - ff));
        if (full != nullptr && n < rows)
          full[(cpos * rows + n) * (int64_t)(C * R3) + ff] = pw;
      }
    }
#pragma unroll
    for (int s = 8; s >= 1; s >>= 1) best = umax64(best, shfl_xor64(best, s));
    if (tf == 0 && n < rows) atomicMax(&packed[cpos * rows + n], best);
  }
}

}  // namespace

hipError_t launch_fine_f32(dsgrft_plan p, int64_t nunits, int64_t unit0,
                           float *full, int64_t /*full_cell0*/, hipStream_t s) {
  int64_t tiles = nunits * (p->rows_p / TN) * (p->Cp / TF);
  hipLaunchKernelGGL(k_fine_f32, dim3((unsigned)tiles), dim3(256), 0, s,
                     (const float2 *)p->G, p->F32, p->packed, full, p->Mp,
                     p->rows_p, p->Cp, nunits, unit0, p->R3, p->C, p->rows);
  return hipGetLastError();
}
