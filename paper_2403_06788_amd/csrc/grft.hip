// Single-scale TD-GRFT (Sec. III-A-1, eq. (13)) in FP32:
//   Y_G(n0; i) = sum_m S(m, n0 + off(m; i)) exp(+j 2 pi Num(m; i) / M^3)
// with the range offset taken along each lattice point's own full walk.  The
// lattice points are the same as the DS-GRFT cells (coarse centre + fine
// offset), so the two maps compare cell by cell.
//
// A workgroup takes one coarse cell, FG = 8 consecutive fine cells and 1024
// range rows (four per thread, 256 apart).  For each chunk of 32 pulses the
// FG x 32 offsets and phasors are formed from exact integers (FP64 sincospi,
// rounded to FP32) into LDS, one entry per thread, with each pulse's smallest
// offset lo and largest hi over the group.  The fine cells of a coarse cell
// walk within about a bin of its centre, so at one pulse a group's offsets
// nearly always fall in one or two bins: a thread loads the samples of its
// rows at each bin of [lo, hi] once and every cell takes the load of its own
// bin, rather than one load per cell; the group's phasors of a pulse are
// read together, as wave-uniform LDS values, before its FMAs.  Each cell's sum takes the same
// samples in the same order with the same FMAs as a direct evaluation (a
// sample past the echo's ends is zero).
#include "internal.h"

namespace {

constexpr int FG = 8, MC = 32, RPT = 4, RWG = 256 * RPT, PG = 64 / FG;

__device__ inline unsigned long long umax64(unsigned long long a,
                                            unsigned long long b) {
  return a > b ? a : b;
}

__global__ __launch_bounds__(256, 4) void k_grft(
    const float2 *__restrict__ echo, int64_t cc_begin, int M, int N, int n_begin,
    int rows, int R, int P, int K0, int K1, int K2, int i0, int i1, int i2, Lat L,
    int64_t n_fine, unsigned long long *__restrict__ packed,
    float *__restrict__ full, int64_t full_cell0) {
  __shared__ float2 s_ph[MC * FG];
  __shared__ int s_off[MC * FG];
  __shared__ int s_lo[MC], s_hi[MC];
  const int64_t nfg = (n_fine + FG - 1) / FG;
  const int rb = (rows + RWG - 1) / RWG;
  const int64_t bid = blockIdx.x;
  const int rblk = (int)(bid % rb);
  const int64_t fg = (bid / rb) % nfg;
  const int64_t cpos = bid / (rb * nfg);
  const int64_t k = cc_begin + cpos;
  const int tid = threadIdx.x, lane = tid & 63;
  const int r0 = rblk * RWG + tid;  // rows r0 + 256 j
  const int nvalid = (int)((n_fine - fg * FG) < FG ? (n_fine - fg * FG) : FG);
  const unsigned all = (1u << nvalid) - 1u;

  // the table entry this thread forms: cell tid % FG at pulse m0 + tid / FG
  static_assert(MC * FG == 256, "one table entry per thread");
  const int tq = tid % FG;
  __shared__ int64_t s_lp[3][256];  // its lattice point
  {
    int Ks[3] = {K0, K1, K2}, il[3] = {i0, i1, i2};
    int64_t ic[3], fo[3];
    coarse_centre(Ks, il, R, P, k, ic, R);
    fine_offsets(R, P, fg * FG + (tq < nvalid ? tq : 0), fo, R);
    for (int a = 0; a < 3; ++a) s_lp[a][tid] = ic[a] + fo[a];
  }

  float2 acc[FG][RPT];
#pragma unroll
  for (int q = 0; q < FG; ++q)
#pragma unroll
    for (int j = 0; j < RPT; ++j) acc[q][j] = make_float2(0.f, 0.f);

  // The samples of a thread's rows at offset b of one pulse's row, read
  // through a buffer resource spanning that row: an index outside [0, N)
  // (a negative one taken as a large unsigned, then clamped to N) reads zero.
  auto window = [&](float2 (&w)[RPT], const float2 *row, int b) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float2 *>(row), 0, N * 8, 0x00020000);
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int idx = n_begin + r0 + 256 * j + b;
      const unsigned e = min((unsigned)idx, (unsigned)N);
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(e * 8u), 0, 0);
      w[j] = make_float2(__int_as_float(v[0]), __int_as_float(v[1]));
    }
  };

  for (int m0 = 0; m0 < M; m0 += MC) {
    {
      const int m = m0 + tid / FG;
      int o = 0;
      float2 ph = make_float2(0.f, 0.f);
      if (tq < nvalid && m < M) {
        const int64_t num = lat_num(L, m, s_lp[0][tid], s_lp[1][tid], s_lp[2][tid]);
        o = lat_offset(L, num);
        ph = lat_phasor(L, num);
      }
      s_off[tid] = o;
      s_ph[tid] = ph;
    }
    __syncthreads();
    if (tid < MC) {
      int lo = s_off[tid * FG], hi = lo;
      for (int q = 1; q < nvalid; ++q) {
        lo = min(lo, s_off[tid * FG + q]);
        hi = max(hi, s_off[tid * FG + q]);
      }
      s_lo[tid] = lo;
      s_hi[tid] = hi;
    }
    __syncthreads();
    const int mc = (M - m0) < MC ? (M - m0) : MC;
    for (int mm = 0; mm < mc; ++mm) {
      // lane l holds the offset of (pulse mm - mm % PG + l / FG, cell l % FG)
      const int offl = s_off[(mm / PG) * 64 + lane];
      const int l0 = (mm % PG) * FG;
      const float2 *row = echo + (int64_t)(m0 + mm) * N;
      const int lo = __builtin_amdgcn_readfirstlane(s_lo[mm]);
      const int hi = __builtin_amdgcn_readfirstlane(s_hi[mm]);
      float2 wc[RPT];
      window(wc, row, lo);
      float2 ph[FG];
#pragma unroll
      for (int q = 0; q < FG; ++q) ph[q] = s_ph[mm * FG + q];
      // one pass per bin in [lo, hi], each cell in the pass of its offset
      for (int b = lo; b <= hi; ++b) {
        const unsigned in =
            (unsigned)(__builtin_amdgcn_ballot_w64(lane / FG == mm % PG && offl == b) >> l0) &
            all;
        float2 w[RPT];
        if (b == lo) {
#pragma unroll
          for (int j = 0; j < RPT; ++j) w[j] = wc[j];
        } else {
          window(w, row, b);
        }
#pragma unroll
        for (int q = 0; q < FG; ++q) {
          if ((in >> q) & 1u) {
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
              acc[q][j].x = fmaf(w[j].x, ph[q].x, fmaf(-w[j].y, ph[q].y, acc[q][j].x));
              acc[q][j].y = fmaf(w[j].x, ph[q].y, fmaf(w[j].y, ph[q].x, acc[q][j].y));
            }
          }
        }
      }
    }
    __syncthreads();
  }

  unsigned long long best[RPT] = {};
#pragma unroll
  for (int q = 0; q < FG; ++q) {
    const int64_t f = fg * FG + q;
    if (q < nvalid) {
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int r = r0 + 256 * j;
        const float pw = acc[q][j].x * acc[q][j].x + acc[q][j].y * acc[q][j].y;
        best[j] = umax64(best[j], ((unsigned long long)__float_as_uint(pw) << 32) |
                                      (0xffffffffu - (unsigned)f));
        if (full && r < rows) full[((full_cell0 + cpos) * rows + r) * n_fine + f] = pw;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int r = r0 + 256 * j;
    if (r < rows) atomicMax(&packed[cpos * rows + r], best[j]);
  }
}

}  // namespace

// Cells [cc_begin, cc_begin + n) with n <= batch_cells; packed must be zeroed.
hipError_t launch_grft(dsgrft_plan p, const float2 *echo, int64_t cc_begin,
                       int64_t n, float *full, hipStream_t s) {
  if (p->N > (1 << 27)) return hipErrorInvalidValue;  // byte offsets of a row in 31 bits
  const int64_t nfg = (p->n_fine + FG - 1) / FG;
  const int rb = (p->rows + RWG - 1) / RWG;
  const int64_t blocks = n * nfg * rb;
  hipLaunchKernelGGL(k_grft, dim3((unsigned)blocks), dim3(256), 0, s, echo,
                     cc_begin, p->M, p->N, p->n_begin, p->rows, p->R, p->P,
                     p->K[0], p->K[1], p->K[2], p->ilo[0], p->ilo[1], p->ilo[2],
                     p->lat, p->n_fine, p->packed, full, (int64_t)0);
  return hipGetLastError();
}
