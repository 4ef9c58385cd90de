// Stages a3 + a4, FFT form: the fine search of the GFT (eq. (44)) evaluated
// the way Alg. 2 does it, with a slow-time FFT.
//
// With the coarse walk gathered and de-ramped (stages a1 + a2, FP32 layout
// G[u][m][n]), the fine phase of orders 1 and 2 is
//   exp(+j 2 pi (f1 m / M + f2 m^2 / M^2)),
// so for each fine acceleration offset f2 the fine velocities f1 are bins of
// one inverse DFT of the de-chirped row:
//   Y[f1, f2][n] = sum_m (G[m][n] c_f2[m]) exp(+j 2 pi f1 m / M)
//               = X_f2[f1 mod M],   c_f2[m] = exp(+j 2 pi f2 m^2 / M^2).
// The wanted bins are the RV fine velocities [-HV, RV - HV) taken mod M: the
// R fine velocities of a DS-GRFT cell (RV = R, HV = R/2; when M < R several
// f1 share a bin and get identical values), or for DS-KT-MFP all M baseband
// velocities i1' in [-M/2, M/2) of the folded lattice (RV = M, HV = M/2,
// Prop. 3).  The flat fine index is f = u2 RV + u1.  Order 3 sits in the
// gathered units as in the GEMM form.
//
// FFT of length M = A B (Cooley-Tukey, decimation in time): with
// m = B m1 + m2 and output bin b = c + A d,
//   X[c + A d] = sum_m2 W_B^(m2 d) [ W_M^(m2 c) sum_m1 W_A^(m1 c) x[B m1 + m2] ],
// W_K = exp(+j 2 pi / K).  Pass 1: thread m2 holds x[B m1 + m2] for all m1 in
// registers and runs an A-point FFT there, scales by the twiddles W_M^(m2 c)
// and writes the A results to LDS; pass 2: thread c reads its B values and
// runs a B-point FFT.  A workgroup owns NROW range rows of one unit; each
// row's gathered samples stay in registers for all R chirps, and each thread
// keeps its best (power, -fine) key, merged per row at the end with the same
// 64-bit atomicMax as the GEMM form (ties to the smaller fine index).
// No implicit contraction in this file: the full-map and reduced-map variants
// of a kernel must round identically, so every fused multiply-add is explicit.
#pragma clang fp contract(off)

#include "fft_reg.h"
#include "internal.h"

namespace {

using fftreg::cmulf;
using fftreg::fft_reg;

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

// G: gathered batch [nunits][Mp][rows_p] complex64; chirp [R2][M]; twM [M].
// R2 = R for P >= 2 (f2 = i2 - R/2), 1 for P = 1; C = RV R2.
template <int A, int B>
__global__ __launch_bounds__(256) void k_fine_fft(
    const float2 *__restrict__ G, const float2 *__restrict__ chirp,
    const float2 *__restrict__ twM, unsigned long long *__restrict__ packed,
    float *__restrict__ full, int Mp, int rows, int rows_p, int RV, int HV, int R2,
    int64_t unit0, int R3, int C) {
  constexpr int M = A * B;
  constexpr int T = A > B ? A : B;  // threads per row
  constexpr int NROW = 256 / T;
  constexpr int ZS = A + 1;         // padded LDS row of pass-1 results
  __shared__ float2 s_tw[M];
  __shared__ float2 s_z[NROW * B * ZS];
  const int tid = threadIdx.x;
  const int rl = tid / T, q = tid % T;
  const int bpu = rows_p / NROW;
  const int64_t u = blockIdx.x / bpu;
  const int n = (int)(blockIdx.x % bpu) * NROW + rl;
  for (int i = tid; i < M; i += 256) s_tw[i] = twM[i];

  float2 g[A];
  if (q < B) {
#pragma unroll
    for (int m1 = 0; m1 < A; ++m1)
      g[m1] = G[((int64_t)u * Mp + B * m1 + q) * rows_p + n];
  }
  __syncthreads();

  const int64_t ug = unit0 + u;
  const int64_t cpos = ug / R3;
  const unsigned fbase = (unsigned)((ug % R3) * C);
  unsigned long long best = 0ull;
  float2 *zrow = s_z + rl * B * ZS;
  for (int i2 = 0; i2 < R2; ++i2) {
    if (q < B) {
      const float2 *ch = chirp + (int64_t)i2 * M;
      float2 x[A];
#pragma unroll
      for (int m1 = 0; m1 < A; ++m1) x[m1] = cmulf(g[m1], ch[B * m1 + q]);
      fft_reg<A>(x);
#pragma unroll
      for (int c = 0; c < A; ++c) zrow[q * ZS + c] = cmulf(x[c], s_tw[(q * c) & (M - 1)]);
    }
    __syncthreads();
    if (q < A) {
      float2 y[B];
#pragma unroll
      for (int d = 0; d < B; ++d) y[d] = zrow[d * ZS + q];
      fft_reg<B>(y);
#pragma unroll
      for (int d = 0; d < B; ++d) {
        const int b = q + A * d;
        const float pw = fmaf(y[d].x, y[d].x, y[d].y * y[d].y);
        // fine velocity indices u1 in [0, RV) with (u1 - HV) = b (mod M)
        for (int u1 = (b + HV) % M; u1 < RV; u1 += M) {
          const unsigned ff = fbase + (unsigned)(i2 * RV + u1);
          best = umax64(best, ((unsigned long long)__float_as_uint(pw) << 32) |
                                  (0xffffffffu - ff));
          if (full != nullptr && n < rows)
            full[(cpos * rows + n) * (int64_t)(C * R3) + ff] = pw;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 1; s < T; s <<= 1) best = umax64(best, shfl_xor64(best, s));
  if (q == 0 && n < rows) atomicMax(&packed[cpos * rows + n], best);
}

// Orders LDS accesses of one wavefront: its lanes exchange data through a
// private LDS region, and LDS operations of a wavefront complete in order, so
// a wavefront-scope fence is all the ordering needed (no workgroup barrier).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wavefront-per-row form for M = 64 P (P = 8, 16, 32): each wavefront owns a
// range row, each lane P of its pulses.  With m = 64 a + l (lane l) and
// output bin k = k1 + P (k2a + 8 k2b),
//   X[k] = sum_l2 W_8^(l2 k2b) W_64^(l2 k2a)
//            sum_l1 W_8^(l1 k2a) W_M^(l k1) sum_a x[64 a + l] W_P^(a k1),
// l = 8 l1 + l2: pass 1 is a P-point FFT over a in the lane's registers
// followed by the twiddles W_M^(l k1) (from LDS); pass 2, on lane 8 kq + l2,
// the 8-point FFTs over l1 for k1 = kq + 8 j and the twiddles W_64^(l2 k2a);
// pass 3, on lane 8 kq + k2a, the 8-point FFTs over l2.  The two exchanges go
// through the wavefront's LDS rows: exchange 1 puts Z[l][k1] in row
// 8 (k1 / 8) + l / 8 (length 72) at 8 (k1 % 8) + l % 8, exchange 2 puts
// V[k1][l2][k2a] in row 8 j + k2a (length 65) at 8 kq + l2; every access of
// both is conflict-free (contiguous on one side, padded rows on the other).
// FULL (RV = M, HV = M/2) maps bin k to u1 = k xor M/2 (one fine index per
// bin, no range test).  PRUNE (HV <= M/8 and RV - HV <= M/8, as for the R =
// 100 fine velocities of a DS-GRFT cell at M >= 512): every wanted bin has
// k2b = 0 (bins below M/8) or k2b = 7 (bins from 7M/8), so pass 3 forms only
// those two outputs of each 8-point transform, X0 = sum v and
// X7 = sum v exp(-j 2 pi l2 / 8), and the power and range tests cover 2 of 8.
template <int P, int NW, bool FULL, bool WFULL, bool PRUNE>
__global__ __launch_bounds__(64 * NW) void k_fine_fft_w(
    const float2 *__restrict__ G, const float2 *__restrict__ chirp,
    const float2 *__restrict__ twM, unsigned long long *__restrict__ packed,
    float *__restrict__ full, int Mp, int rows, int rows_p, int RV, int HV, int R2,
    int64_t unit0, int R3, int C) {
  constexpr int M = 64 * P;
  constexpr int NJ = P / 8;
  constexpr int ROW1 = 72, ROW2 = 65;
  constexpr int XS = P * ROW1;
  static_assert(P % 8 == 0 && P <= 32, "points per lane");
  static_assert(!(FULL && PRUNE), "all bins or the outer eighths");
  constexpr int NK = PRUNE ? 2 : 8;  // outputs per 8-point transform of pass 3
  __shared__ float2 s_tw[M];            // [k1][l] = W_M^(l k1)
  __shared__ float2 s_x[NW * XS];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int bpu = rows_p / NW;
  const int64_t u = blockIdx.x / bpu;
  const int n = (int)(blockIdx.x % bpu) * NW + w;
  for (int i = tid; i < M; i += 64 * NW) s_tw[i] = twM[((i & 63) * (i >> 6)) & (M - 1)];
  float2 g[P];
#pragma unroll
  for (int a = 0; a < P; ++a) g[a] = G[((int64_t)u * Mp + 64 * a + lane) * rows_p + n];
  // W_64^(l2 k2a) for this lane's l2 in pass 2
  float2 t2[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) t2[k] = twM[(P * (lane & 7) * k) & (M - 1)];
  __syncthreads();
  // at M = 1024, this lane's W_M^(l k1) for k1 < NTR held in registers (all
  // of them in the pruned variant, half in the all-bins one, as their
  // registers allow at three waves per SIMD); the rest, and every twiddle at
  // other M, read from LDS for every chirp
  constexpr int NTR = P != 16 ? 0 : PRUNE ? P : FULL ? P / 2 : 0;
  float2 t1[NTR > 0 ? NTR : 1];
#pragma unroll
  for (int k1 = 0; k1 < NTR; ++k1) t1[k1] = s_tw[k1 * 64 + lane];

  const int64_t ug = unit0 + u;
  const int64_t cpos = ug / R3;
  const unsigned fbase = (unsigned)((ug % R3) * C);
  float2 *xb = s_x + w * XS;
  const int kq = lane >> 3, lo3 = lane & 7;
  // Fast argmax: each lane keeps its largest power over the wanted bins and
  // the first chirp reaching it; after the last chirp the wavefront takes the
  // best (power, smallest chirp) and runs that chirp once more through the
  // same loop body with the exact per-bin keys (power bits, ~fine index), so
  // ties still go to the smaller fine index.  The full-map variant (WFULL)
  // and short chirp counts use the per-bin keys on every chirp.
  if (FULL) {
    RV = M;
    HV = M / 2;
  }
  const bool direct = WFULL || R2 < 4;
  float bp = 0.f;
  int bi = 0;
  unsigned long long best = 0ull;
  const int iters = direct ? R2 : R2 + 1;
  for (int it = 0; it < iters; ++it) {
    const bool fin = !direct && it == R2;
    int i2 = it;
    if (fin) {
      unsigned long long kb = ((unsigned long long)__float_as_uint(bp) << 32) |
                              (0xffffffffu - (unsigned)bi);
#pragma unroll
      for (int s = 1; s < 64; s <<= 1) kb = umax64(kb, shfl_xor64(kb, s));
      i2 = __builtin_amdgcn_readfirstlane((int)(0xffffffffu - (unsigned)kb));
    }
    const float2 *ch = chirp + (int64_t)i2 * M;
    float2 x[P];
#pragma unroll
    for (int a = 0; a < P; ++a) x[a] = cmulf(g[a], ch[64 * a + lane]);
    fft_reg<P>(x);
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) {
      const float2 z = k1 ? cmulf(x[k1], k1 < NTR ? t1[k1 < NTR ? k1 : 0] : s_tw[k1 * 64 + lane])
                          : x[0];
      xb[((k1 >> 3) * 8 + kq) * ROW1 + 8 * (k1 & 7) + lo3] = z;
    }
    wave_lds_sync();
    float2 v[NJ][8];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
#pragma unroll
      for (int l1 = 0; l1 < 8; ++l1) v[j][l1] = xb[(j * 8 + l1) * ROW1 + lane];
    }
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      fft_reg<8>(v[j]);
#pragma unroll
      for (int k = 1; k < 8; ++k) v[j][k] = cmulf(v[j][k], t2[k]);
#pragma unroll
      for (int k = 0; k < 8; ++k) xb[(j * 8 + k) * ROW2 + lane] = v[j][k];
    }
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
#pragma unroll
      for (int l2 = 0; l2 < 8; ++l2) v[j][l2] = xb[(j * 8 + lo3) * ROW2 + 8 * kq + l2];
    }
    wave_lds_sync();
    // pass 3; output e of transform j is bin k2b = kb(e)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      if constexpr (PRUNE) {
        constexpr float h = 0.70710678118654752f;  // sqrt(1/2)
        float2 a[4], b[4];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          a[l] = make_float2(v[j][l].x + v[j][l + 4].x, v[j][l].y + v[j][l + 4].y);
          b[l] = make_float2(v[j][l].x - v[j][l + 4].x, v[j][l].y - v[j][l + 4].y);
        }
        const float2 c = make_float2(b[1].x - b[3].x, b[1].y - b[3].y);
        const float2 d = make_float2(b[1].x + b[3].x, b[1].y + b[3].y);
        v[j][0] = make_float2((a[0].x + a[2].x) + (a[1].x + a[3].x),
                              (a[0].y + a[2].y) + (a[1].y + a[3].y));
        v[j][1] = make_float2(fmaf(h, c.x + d.y, b[0].x + b[2].y),
                              fmaf(h, c.y - d.x, b[0].y - b[2].x));
      } else {
        fft_reg<8>(v[j]);
      }
    }
    auto kb = [](int e) { return PRUNE ? 7 * e : e; };
    if (!direct && !fin) {
      float cm = 0.f;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
#pragma unroll
        for (int e = 0; e < NK; ++e) {
          const float pw = fmaf(v[j][e].x, v[j][e].x, v[j][e].y * v[j][e].y);
          if (FULL) {
            cm = fmaxf(cm, pw);
          } else {
            const int b = kq + 8 * j + P * (lo3 + 8 * kb(e));
            cm = ((b + HV) % M < RV) ? fmaxf(cm, pw) : cm;
          }
        }
      }
      if (cm > bp) {
        bp = cm;
        bi = i2;
      }
    } else {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
#pragma unroll
        for (int e = 0; e < NK; ++e) {
          const int b = kq + 8 * j + P * (lo3 + 8 * kb(e));
          const float pw = fmaf(v[j][e].x, v[j][e].x, v[j][e].y * v[j][e].y);
          for (int u1 = FULL ? (b ^ (M / 2)) : (b + HV) % M; u1 < RV; u1 += M) {
            const unsigned ff = fbase + (unsigned)(i2 * RV + u1);
            best = umax64(best, ((unsigned long long)__float_as_uint(pw) << 32) |
                                    (0xffffffffu - ff));
            if (WFULL && n < rows) full[(cpos * rows + n) * (int64_t)(C * R3) + ff] = pw;
          }
        }
      }
    }
  }
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) best = umax64(best, shfl_xor64(best, s));
  if (lane == 0 && n < rows) atomicMax(&packed[cpos * rows + n], best);
}

__global__ void k_fft_tables(int M, int R, int R2, int P, Lat L, float2 *twM,
                             float2 *chirp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < M) {
    double s, c;
    sincospi(2.0 * (double)t / (double)M, &s, &c);
    twM[t] = make_float2((float)c, (float)s);
  }
  if (t < (int64_t)R2 * M) {
    const int i2 = (int)(t / M), m = (int)(t % M);
    const int64_t f2 = (P >= 2) ? (int64_t)(i2 - R / 2) : 0;
    chirp[t] = lat_phasor(L, lat_num(L, m, 0, f2, 0));
  }
}

template <int A, int B>
hipError_t launch_ab(dsgrft_plan p, int64_t nunits, int64_t unit0, float *full,
                     hipStream_t s) {
  constexpr int T = A > B ? A : B;
  constexpr int NROW = 256 / T;
  const int64_t blocks = nunits * (p->rows_p / NROW);
  const int R2 = p->P >= 2 ? p->R : 1;
  hipLaunchKernelGGL((k_fine_fft<A, B>), dim3((unsigned)blocks), dim3(256), 0, s,
                     (const float2 *)p->G, p->fft_chirp, p->fft_tw,
                     p->packed, full, p->Mp, p->rows, p->rows_p, p->S0, p->S0 / 2, R2,
                     unit0, p->R3, p->C);
  return hipGetLastError();
}

template <int P, int NW>
hipError_t launch_w(dsgrft_plan p, int64_t nunits, int64_t unit0, float *full,
                    hipStream_t s) {
  const int64_t blocks = nunits * (p->rows_p / NW);
  const int R2 = p->P >= 2 ? p->R : 1;
  const bool fullbins = p->S0 == p->M;
  const int M = 64 * P, hv = p->S0 / 2;
  const bool prune = !fullbins && hv <= M / 8 && p->S0 - hv <= M / 8;
  auto kern = fullbins ? (full ? k_fine_fft_w<P, NW, true, true, false>
                               : k_fine_fft_w<P, NW, true, false, false>)
              : prune  ? (full ? k_fine_fft_w<P, NW, false, true, true>
                               : k_fine_fft_w<P, NW, false, false, true>)
                       : (full ? k_fine_fft_w<P, NW, false, true, false>
                               : k_fine_fft_w<P, NW, false, false, false>);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * NW), 0, s, (const float2 *)p->G,
                     p->fft_chirp, p->fft_tw, p->packed, full, p->Mp, p->rows, p->rows_p,
                     p->S0, p->S0 / 2, R2, unit0, p->R3, p->C);
  return hipGetLastError();
}

}  // namespace

bool fft_form_supported(int M) {
  return M >= 64 && M <= 2048 && (M & (M - 1)) == 0;
}

size_t fft_table_elems(int M, int R, int P) {
  return (size_t)M + (size_t)(P >= 2 ? R : 1) * M;
}

hipError_t launch_fft_tables(dsgrft_plan p, hipStream_t s) {
  const int R2 = p->P >= 2 ? p->R : 1;
  const int64_t n = (int64_t)R2 * p->M;
  hipLaunchKernelGGL(k_fft_tables, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     p->M, p->R, R2, p->P, p->lat, p->fft_tw, p->fft_chirp);
  return hipGetLastError();
}

hipError_t launch_fine_fft(dsgrft_plan p, int64_t nunits, int64_t unit0,
                           float *full, hipStream_t s) {
  switch (p->M) {
    case 64: return launch_ab<8, 8>(p, nunits, unit0, full, s);
    case 128: return launch_ab<16, 8>(p, nunits, unit0, full, s);
    case 256: return launch_ab<16, 16>(p, nunits, unit0, full, s);
    case 512: return launch_w<8, 4>(p, nunits, unit0, full, s);
    case 1024: return launch_w<16, 4>(p, nunits, unit0, full, s);
    case 2048: return launch_w<32, 2>(p, nunits, unit0, full, s);
    default: return hipErrorInvalidValue;
  }
}
