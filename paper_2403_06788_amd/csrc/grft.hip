// Single-scale TD-GRFT (Sec. III-A-1, eq. (13)) in FP32:
//   Y_G(n0; i) = sum_m S(m, n0 + off(m; i)) exp(+j 2 pi Num(m; i) / M^3)
// with the range offset taken along each lattice point's own full walk.  The
// lattice points are the same as the DS-GRFT cells (coarse centre + fine
// offset), so the two maps compare cell by cell.
//
// A workgroup takes one coarse cell, 8 consecutive fine cells and 256 range
// rows.  For each chunk of 32 pulses the 8 x 32 offsets and phasors are formed
// from exact integers (FP64 sincospi, rounded to FP32) into LDS; each thread
// then accumulates its row for the 8 cells.  The echo reads of one pulse are
// contiguous across the workgroup.
#include "internal.h"

namespace {

constexpr int FG = 8, MC = 32;

__device__ inline unsigned long long umax64(unsigned long long a,
                                            unsigned long long b) {
  return a > b ? a : b;
}

__global__ __launch_bounds__(256) void k_grft(
    const float2 *__restrict__ echo, int64_t cc_begin, int M, int N, int n_begin,
    int rows, int R, int P, int K0, int K1, int K2, int i0, int i1, int i2, Lat L,
    int64_t n_fine, unsigned long long *__restrict__ packed,
    float *__restrict__ full, int64_t full_cell0) {
  __shared__ int s_off[FG][MC];
  __shared__ float2 s_ph[FG][MC];
  const int64_t nfg = (n_fine + FG - 1) / FG;
  const int rb = (rows + 255) / 256;
  const int64_t bid = blockIdx.x;
  const int rblk = (int)(bid % rb);
  const int64_t fg = (bid / rb) % nfg;
  const int64_t cpos = bid / (rb * nfg);
  const int64_t k = cc_begin + cpos;
  const int tid = threadIdx.x;
  const int r = rblk * 256 + tid;

  int Ks[3] = {K0, K1, K2}, il[3] = {i0, i1, i2};
  int64_t ic[3];
  coarse_centre(Ks, il, R, P, k, ic, R);

  float2 acc[FG];
#pragma unroll
  for (int q = 0; q < FG; ++q) acc[q] = make_float2(0.f, 0.f);

  for (int m0 = 0; m0 < M; m0 += MC) {
    {
      const int q = tid / MC, mm = tid % MC;
      const int64_t f = fg * FG + q;
      const int m = m0 + mm;
      int o = 0;
      float2 ph = make_float2(0.f, 0.f);
      if (f < n_fine && m < M) {
        int64_t fo[3];
        fine_offsets(R, P, f, fo, R);
        const int64_t num = lat_num(L, m, ic[0] + fo[0], ic[1] + fo[1], ic[2] + fo[2]);
        o = lat_offset(L, num);
        ph = lat_phasor(L, num);
      }
      s_off[q][mm] = o;
      s_ph[q][mm] = ph;
    }
    __syncthreads();
    if (r < rows) {
      const int mend = (M - m0) < MC ? (M - m0) : MC;
      for (int mm = 0; mm < mend; ++mm) {
        const float2 *row = echo + (int64_t)(m0 + mm) * N;
#pragma unroll
        for (int q = 0; q < FG; ++q) {
          const int idx = n_begin + r + s_off[q][mm];
          if (idx >= 0 && idx < N) {
            const float2 s = row[idx];
            const float2 ph = s_ph[q][mm];
            acc[q].x = fmaf(s.x, ph.x, fmaf(-s.y, ph.y, acc[q].x));
            acc[q].y = fmaf(s.x, ph.y, fmaf(s.y, ph.x, acc[q].y));
          }
        }
      }
    }
    __syncthreads();
  }
  if (r >= rows) return;
  unsigned long long best = 0ull;
#pragma unroll
  for (int q = 0; q < FG; ++q) {
    const int64_t f = fg * FG + q;
    if (f < n_fine) {
      const float pw = acc[q].x * acc[q].x + acc[q].y * acc[q].y;
      best = umax64(best, ((unsigned long long)__float_as_uint(pw) << 32) |
                              (0xffffffffu - (unsigned)f));
      if (full) full[((full_cell0 + cpos) * rows + r) * n_fine + f] = pw;
    }
  }
  atomicMax(&packed[cpos * rows + r], best);
}

}  // namespace

// Cells [cc_begin, cc_begin + n) with n <= batch_cells; packed must be zeroed.
hipError_t launch_grft(dsgrft_plan p, const float2 *echo, int64_t cc_begin,
                       int64_t n, float *full, hipStream_t s) {
  const int64_t nfg = (p->n_fine + FG - 1) / FG;
  const int rb = (p->rows + 255) / 256;
  const int64_t blocks = n * nfg * rb;
  hipLaunchKernelGGL(k_grft, dim3((unsigned)blocks), dim3(256), 0, s, echo,
                     cc_begin, p->M, p->N, p->n_begin, p->rows, p->R, p->P,
                     p->K[0], p->K[1], p->K[2], p->ilo[0], p->ilo[1], p->ilo[2],
                     p->lat, p->n_fine, p->packed, full, (int64_t)0);
  return hipGetLastError();
}
