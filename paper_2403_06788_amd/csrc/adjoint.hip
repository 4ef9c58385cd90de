// Continuous DS-GRFT objective, its adjoint and off-grid refinement (FP64).
//
// The paper defines the transforms on the search lattice only; the off-grid
// objective is this library's reading.  For theta = (r0, v, a):
//   coarse cell  k_p = clamp(floor((theta_p/d_p - i_lo,p + 1/2) / R)), centre i_c
//   envelope     x_m = r0/dr + off(m; i_c)   (coarse walk, as in mGIFT)
//   interpolant  s~_m(x) = sum_{n<N} s[m][n] sinc(x - n)
//   phase        cyc_m = 2 (v t_m + a t_m^2/2) / lambda, range-reduced in FP64
//   Y = sum_m s~_m(x_m) exp(j 2 pi cyc_m),  J = |Y|^2.
// J equals the DS-GRFT power map at lattice points (sinc of an integer is a
// Kronecker delta).  sinc(x - n) is evaluated as (-1)^(floor(x) - n)
// sinpi(frac(x)) / (pi (x - n)), with a series near zero.
//
// Forward: a workgroup of 256 threads takes CB candidates (2 for the forward
// and gradient pass; 1 for refinement, whose batches are small: few
// candidates per workgroup keep the registers low enough for several waves
// per SIMD and, for a small batch, give enough workgroups); per chunk of
// 256 / CB pulses the per-(candidate, pulse) quantities are formed once into
// LDS; each group of 64 threads then takes every fourth pulse and sweeps its
// range taps for all CB candidates, reusing every echo load CB times.
// Accumulated per thread: Y, dY/dr0 (with sinc'), sum s~ e t and
// sum s~ e t^2 (for dY/dv, dY/da), reduced at the end.
#include "internal.h"

namespace {

constexpr int CB_FWD = 2;  // candidates per workgroup, forward and gradients
constexpr int CB_REF = 1;  // candidates per workgroup, refinement
constexpr int TPB = 256;

struct AdjCtx {
  int M, N, P, R, K0, K1, ilo0, ilo1;
  double dr, prf, lam, st0, st1;
  Lat L;
};

struct Tap {   // per (candidate, pulse)
  double xf, sp, cp, er, ei, t;
  int xi;
  int pad;
};

__device__ inline void centre_of(const AdjCtx &c, double v, double a, int64_t ic[2]) {
  const double th[2] = {v, a};
  const int K[2] = {c.K0, c.K1}, il[2] = {c.ilo0, c.ilo1};
  const double st[2] = {c.st0, c.st1};
  for (int p = 0; p < 2; ++p) {
    if (p >= c.P) {
      ic[p] = 0;
      continue;
    }
    double u = th[p] / st[p];
    double kf = floor((u - (double)il[p] + 0.5) / (double)c.R);
    int64_t k = (int64_t)kf;
    if (kf < 0) k = 0;
    if (kf > K[p] - 1) k = K[p] - 1;
    ic[p] = (int64_t)il[p] + k * c.R + c.R / 2;
  }
}

__device__ inline Tap make_tap(const AdjCtx &c, const double *th, const int64_t *ic,
                               int m) {
  Tap T;
  const int64_t num = lat_num(c.L, m, ic[0], ic[1], 0);
  const double x = th[0] / c.dr + (double)lat_offset(c.L, num);
  const double xi = floor(x);
  T.xi = (int)xi;
  T.xf = x - xi;
  sincospi(T.xf, &T.sp, &T.cp);
  const double t = (double)m / c.prf;
  const double cyc = 2.0 * (th[1] * t + th[2] * t * t / 2.0) / c.lam;
  const double fr = cyc - floor(cyc);
  sincospi(2.0 * fr, &T.ei, &T.er);
  T.t = t;
  T.pad = 0;
  return T;
}

// 1/d in FP64 for 1e-4 <= |d| < 2^24: single-precision seed and two Newton
// steps (relative error ~2^-92, below FP64 rounding).
__device__ inline double recip(double d) {
  double r = (double)__builtin_amdgcn_rcpf((float)d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

// 1/a, 1/b, 1/c, 1/d from one reciprocal (Montgomery's batch inversion):
// with ab = a b, cd = c d and q = 1/(ab cd), 1/a = b cd q, 1/b = a cd q,
// 1/c = d ab q, 1/d = c ab q; error a few FP64 ulps.  Callers pass
// 1e-4 <= |x| < 2^24 for values at least 64 apart, so the product lies in
// [40, 2^96], inside the normal range of recip's single-precision seed.
__device__ inline void recip4(double a, double b, double c, double d, double &ra,
                              double &rb, double &rc, double &rd) {
  const double ab = a * b, cd = c * d;
  const double q = recip(ab * cd);
  const double qab = q * ab, qcd = q * cd;
  ra = qcd * b;
  rb = qcd * a;
  rc = qab * d;
  rd = qab * c;
}

// A/a, A/b, A/c, A/d the same way, with A folded into the one reciprocal.
__device__ inline void recip4_scaled(double A, double a, double b, double c, double d,
                                     double &wa, double &wb, double &wc, double &wd) {
  const double ab = a * b, cd = c * d;
  const double q = A * recip(ab * cd);
  const double qab = q * ab, qcd = q * cd;
  wa = qcd * b;
  wb = qcd * a;
  wc = qab * d;
  wd = qab * c;
}

// sinc(d) and d sinc(d)/dd near d = 0 (|d| < 1e-4), by their series.
__device__ inline void sinc_series(double d, double &w, double &dw) {
  const double pd = M_PI * d;
  w = 1.0 - pd * pd / 6.0;
  dw = -(M_PI * M_PI) * d / 3.0 + (M_PI * M_PI * M_PI * M_PI) * d * d * d / 30.0;
}

__device__ inline double block_sum(double v, double *red) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < TPB / 64; ++w) s += red[w];
  return s;
}

// Computes, for the candidates s_th[0..nb) (in LDS), the 8 complex sums (Y,
// dY/dr0, sum s~ e t, sum s~ e t^2) into out[CB][8] (all threads receive
// them).
template <int CB>
__device__ void eval_block(const AdjCtx &c, const float2 *__restrict__ echo,
                           const double (*s_th)[3], int nb, double (*out)[8],
                           Tap *s_tap, double *red) {
  constexpr int MCH = TPB / CB;  // pulses per table chunk
  double acc[CB][8];
#pragma unroll
  for (int b = 0; b < CB; ++b)
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[b][q] = 0.0;
  const int tid = threadIdx.x;
  for (int m0 = 0; m0 < c.M; m0 += MCH) {
    __syncthreads();
    {
      const int b = tid / MCH, mm = tid % MCH;   // CB * MCH == TPB
      const int m = m0 + mm;
      if (b < nb && m < c.M) {
        const double th[3] = {s_th[b][0], s_th[b][1], s_th[b][2]};
        int64_t ic[2];
        centre_of(c, th[1], th[2], ic);
        s_tap[tid] = make_tap(c, th, ic, m);
      }
    }
    __syncthreads();
    const int mend = (c.M - m0) < MCH ? (c.M - m0) : MCH;
    // pulse group pg = tid / 64 takes every fourth pulse of the chunk; its 64
    // lanes sweep the range taps n = lane + 64 j of that pulse.  The partial
    // sums are linear in the taps, so each thread multiplies its own share by
    // the pulse phasor and the block reduction at the end completes them.
    const int pg = tid >> 6, lane = tid & 63;
    for (int mm = pg; mm < mend; mm += TPB / 64) {
      const float2 *row = echo + (int64_t)(m0 + mm) * c.N;
      // with the tap stride 64 even, the sign (-1)^(xi - n) of
      // sin(pi (x - n)) = (-1)^(xi - n) sin(pi xf) is fixed per thread, and
      // d = x - n steps by exactly -64.
      double sr[CB], si[CB], dr_[CB], di[CB], A[CB], Bc[CB];
      double dc[CB];     // d of this step's first tap, lowered by 256 per step
      bool far_ok[CB];   // every |d| of the sweep below 2^24 (recip4's range)
      int jnear[CB];     // the step j whose taps hold |d| < 1e-4, or -1
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        sr[b] = si[b] = dr_[b] = di[b] = 0.0;
        const Tap &T = s_tap[b * MCH + mm];
        const double sg = ((T.xi - lane) & 1) ? -1.0 : 1.0;
        A[b] = sg * T.sp * (1.0 / M_PI);
        Bc[b] = sg * T.cp;
        const double d0 = (double)(T.xi - lane) + T.xf;
        dc[b] = d0;
        far_ok[b] = fabs(d0) + (double)c.N + 256.0 < 16777216.0;
        // taps are 64 apart, so only tap k = round(d0 / 64) can come within
        // 1e-4 of zero; it sits in step j = 4 floor(k / 4)
        const double ks = floor(d0 * (1.0 / 64.0) + 0.5);
        jnear[b] = (ks >= 0.0 && ks < 1e9 && fabs(d0 - 64.0 * ks) < 1e-4) ? ((int)ks & ~3) : -1;
      }
      // four taps (n, n + 64, n + 128, n + 192) per step, their reciprocals
      // from one (recip4); taps 0, 2 and 1, 3 feed separate accumulators, so
      // that two FMA chains per sum advance independently; summed after the
      // sweep.  Taps at or beyond N carry a zero sample.
      double sr2[CB], si2[CB], dr2[CB], di2[CB];
#pragma unroll
      for (int b = 0; b < CB; ++b) sr2[b] = si2[b] = dr2[b] = di2[b] = 0.0;
      // Samples are loaded one step ahead, so that the four loads of a step
      // are issued together and their latency overlaps the previous step's
      // arithmetic.  While every lane's four taps lie below N (a condition
      // uniform over the wavefront) the loads are plain; near the end they
      // come from a clamped (always valid) index and the taps at or past N
      // are zeroed where they are used.
      auto load = [&](int nn) { return row[nn < c.N ? nn : c.N - 1]; };
      auto all_in = [&](int n_lane0) { return n_lane0 + 63 + 192 < c.N; };
      float2 cur[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) cur[t] = load(lane + 64 * t);
      int j = 0;
      for (int n = lane; n < c.N; n += 256, j += 4) {
        const int n_lane0 = n - lane;
        double sx[4], sy[4];
        if (all_in(n_lane0)) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            sx[t] = (double)cur[t].x;
            sy[t] = (double)cur[t].y;
          }
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const bool in = n + 64 * t < c.N;
            sx[t] = in ? (double)cur[t].x : 0.0;
            sy[t] = in ? (double)cur[t].y : 0.0;
          }
        }
        if (all_in(n_lane0 + 256)) {
          const float2 *nxt = row + n + 256;
#pragma unroll
          for (int t = 0; t < 4; ++t) cur[t] = nxt[64 * t];
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) cur[t] = load(n + 256 + 64 * t);
        }
#pragma unroll
        for (int b = 0; b < CB; ++b) {
          if (b < nb) {
            double w[4], dw[4], d[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) d[t] = dc[b] - 64.0 * t;
            if (j != jnear[b] && far_ok[b]) {
              double r[4];
              recip4(d[0], d[1], d[2], d[3], r[0], r[1], r[2], r[3]);
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                w[t] = A[b] * r[t];
                dw[t] = (Bc[b] - w[t]) * r[t];
              }
            } else {
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                if (fabs(d[t]) < 1e-4) {
                  sinc_series(d[t], w[t], dw[t]);
                } else {
                  const double r = recip(d[t]);
                  w[t] = A[b] * r;
                  dw[t] = (Bc[b] - w[t]) * r;
                }
              }
            }
#pragma unroll
            for (int t = 0; t < 4; t += 2) {
              sr[b] = fma(sx[t], w[t], sr[b]);
              si[b] = fma(sy[t], w[t], si[b]);
              dr_[b] = fma(sx[t], dw[t], dr_[b]);
              di[b] = fma(sy[t], dw[t], di[b]);
              sr2[b] = fma(sx[t + 1], w[t + 1], sr2[b]);
              si2[b] = fma(sy[t + 1], w[t + 1], si2[b]);
              dr2[b] = fma(sx[t + 1], dw[t + 1], dr2[b]);
              di2[b] = fma(sy[t + 1], dw[t + 1], di2[b]);
            }
            dc[b] -= 256.0;
          }
        }
      }
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        sr[b] += sr2[b];
        si[b] += si2[b];
        dr_[b] += dr2[b];
        di[b] += di2[b];
      }
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        if (b < nb) {
          const Tap &T = s_tap[b * MCH + mm];
          // (sr + j si) * (er + j ei)
          const double yr = sr[b] * T.er - si[b] * T.ei;
          const double yi = sr[b] * T.ei + si[b] * T.er;
          const double gr = dr_[b] * T.er - di[b] * T.ei;
          const double gi = dr_[b] * T.ei + di[b] * T.er;
          acc[b][0] += yr;
          acc[b][1] += yi;
          acc[b][2] += gr;
          acc[b][3] += gi;
          acc[b][4] += yr * T.t;
          acc[b][5] += yi * T.t;
          acc[b][6] += yr * T.t * T.t;
          acc[b][7] += yi * T.t * T.t;
        }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < CB; ++b)
    for (int q = 0; q < 8; ++q) out[b][q] = block_sum(acc[b][q], red);
}

// saved[b] = (Y, dY/dr0, dY/dv, dY/da) as complex128
__device__ inline void finish(const AdjCtx &c, const double *o, double *sv) {
  sv[0] = o[0];
  sv[1] = o[1];
  sv[2] = o[2] / c.dr;
  sv[3] = o[3] / c.dr;
  // dY/dv = j 2 pi (2/lambda) sum s~ e t ; j (x + j y) = -y + j x
  const double kv = 2.0 * M_PI * 2.0 / c.lam, ka = 2.0 * M_PI / c.lam;
  sv[4] = -kv * o[5];
  sv[5] = kv * o[4];
  sv[6] = -ka * o[7];
  sv[7] = ka * o[6];
}

template <int CB>
__global__ __launch_bounds__(TPB, 3) void k_adj_fwd(AdjCtx c, const float2 *__restrict__ echo,
                                                 const double *__restrict__ theta, int B,
                                                 double *__restrict__ J,
                                                 double *__restrict__ saved) {
  __shared__ Tap s_tap[TPB];
  __shared__ double red[TPB / 64];
  __shared__ double s_th[CB][3];
  const int b0 = blockIdx.x * CB;
  const int nb = (B - b0) < CB ? (B - b0) : CB;
  if (threadIdx.x < CB * 3) {
    const int b = threadIdx.x / 3, q = threadIdx.x % 3;
    s_th[b][q] = (b < nb) ? theta[(b0 + b) * 3 + q] : 0.0;
  }
  double out[CB][8];
  eval_block<CB>(c, echo, s_th, nb, out, s_tap, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      if (b < nb) {
        double sv[8];
        finish(c, out[b], sv);
        J[b0 + b] = sv[0] * sv[0] + sv[1] * sv[1];
        if (saved)
#pragma unroll
          for (int q = 0; q < 8; ++q) saved[(int64_t)(b0 + b) * 8 + q] = sv[q];
      }
    }
  }
}

__global__ void k_adj_theta(const double *__restrict__ saved,
                            const double *__restrict__ gJ, int B,
                            double *__restrict__ gt) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double *s = saved + (int64_t)b * 8;
  const double g = gJ ? gJ[b] : 1.0;
  for (int p = 0; p < 3; ++p)  // dJ = 2 Re(conj(Y) dY)
    gt[b * 3 + p] = g * 2.0 * (s[0] * s[2 + 2 * p] + s[1] * s[3 + 2 * p]);
}

struct BTap {  // per candidate for one pulse: sinc data and 2 gJ Y conj(e)
  double xf, sp, cr, ci;
  int xi;
  int pad;
};

// grad_s[m][n] = sum_b sinc(x_bm - n) * (2 gJ_b Y_b conj(e_bm)).  One
// workgroup of 2 x 256 threads per (pulse, 2048-bin slab): each half sums
// over its half of every 512-candidate chunk (staged in LDS) for the same
// 2048 bins, and the halves' sums are added at the end (half 0 + half 1, a
// fixed order); two halves double the waves per SIMD of a one-pulse grid.
constexpr int ECHO_TPB = 2 * TPB;

__global__ __launch_bounds__(ECHO_TPB) void k_adj_echo(AdjCtx c, const double *__restrict__ theta,
                                                       int B, const double *__restrict__ saved,
                                                       const double *__restrict__ gJ,
                                                       float2 *__restrict__ ge) {
  constexpr int PER = 8;
  __shared__ BTap s_b[ECHO_TPB];
  __shared__ double s_part[2 * PER][TPB];
  const int slabs = (c.N + TPB * PER - 1) / (TPB * PER);
  const int m = blockIdx.x / slabs;
  const int n0 = (blockIdx.x % slabs) * TPB * PER;
  const int tid = threadIdx.x, half = tid / TPB, t0 = tid % TPB;
  double ar[PER], ai[PER];
  for (int q = 0; q < PER; ++q) ar[q] = ai[q] = 0.0;
  for (int bb = 0; bb < B; bb += ECHO_TPB) {
    __syncthreads();
    const int b = bb + tid;
    if (b < B) {
      double th[3] = {theta[b * 3], theta[b * 3 + 1], theta[b * 3 + 2]};
      int64_t ic[2];
      centre_of(c, th[1], th[2], ic);
      Tap T = make_tap(c, th, ic, m);
      const double g = 2.0 * (gJ ? gJ[b] : 1.0);
      const double yr = saved[(int64_t)b * 8], yi = saved[(int64_t)b * 8 + 1];
      // 2 gJ Y conj(e)
      BTap q;
      q.xf = T.xf;
      q.sp = T.sp;
      q.xi = T.xi;
      q.pad = 0;
      q.cr = g * (yr * T.er + yi * T.ei);
      q.ci = g * (yi * T.er - yr * T.ei);
      s_b[tid] = q;
    }
    __syncthreads();
    const int kb = half * TPB;
    const int kend = (B - bb - kb) < TPB ? (B - bb - kb) : TPB;
    for (int k = 0; k < kend; ++k) {
      const BTap q = s_b[kb + k];
      // n = n0 + t0 + TPB e with n0 and TPB even: fixed sign per thread
      const double sg = ((q.xi - t0) & 1) ? -1.0 : 1.0;
      const double A = sg * q.sp * (1.0 / M_PI);
      const double d0 = (double)(q.xi - n0 - t0) + q.xf;
      // weights four at a time (recip4_scaled) unless the sweep leaves its
      // range or the group holds the one output e = round(d0 / TPB) whose
      // distance can come within 1e-4 of zero
      const bool far_ok = fabs(d0) + (double)(TPB * PER) < 16777216.0;
      const double es = floor(d0 * (1.0 / TPB) + 0.5);
      const int enear =
          (es >= 0.0 && es < PER && fabs(d0 - TPB * es) < 1e-4) ? ((int)es & ~3) : -1;
#pragma unroll
      for (int e0 = 0; e0 < PER; e0 += 4) {
        double d[4], w[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) d[t] = d0 - (double)(TPB * (e0 + t));
        if (e0 != enear && far_ok) {
          recip4_scaled(A, d[0], d[1], d[2], d[3], w[0], w[1], w[2], w[3]);
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            double dw;
            if (fabs(d[t]) < 1e-4) sinc_series(d[t], w[t], dw);
            else w[t] = A * recip(d[t]);
          }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          ar[e0 + t] = fma(w[t], q.cr, ar[e0 + t]);
          ai[e0 + t] = fma(w[t], q.ci, ai[e0 + t]);
        }
      }
    }
  }
  __syncthreads();
  if (half == 1)
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      s_part[2 * e][t0] = ar[e];
      s_part[2 * e + 1][t0] = ai[e];
    }
  __syncthreads();
  if (half == 0)
    for (int e = 0; e < PER; ++e) {
      const int n = n0 + t0 + TPB * e;
      if (n < c.N)
        ge[(int64_t)m * c.N + n] =
            make_float2((float)(ar[e] + s_part[2 * e][t0]), (float)(ai[e] + s_part[2 * e + 1][t0]));
    }
}

// Refinement: per candidate, normalised-gradient steps with a trust radius in
// (range bin, fine velocity step, fine acceleration step) units; a step is
// kept if J does not decrease (radius doubled, at most 2), otherwise the
// radius is halved.  The fine indices stay inside the starting coarse cell,
// r0 inside [0, N-1] bins.
template <int CB>
__global__ __launch_bounds__(TPB, 3) void k_refine(AdjCtx c, const float2 *__restrict__ echo,
                                                double *__restrict__ theta, int B, int iters,
                                                double *__restrict__ Jout) {
  __shared__ Tap s_tap[TPB];
  __shared__ double red[TPB / 64];
  __shared__ double s_th[CB][3];
  const int b0 = blockIdx.x * CB;
  const int nb = (B - b0) < CB ? (B - b0) : CB;
  // every thread keeps the same per-candidate state; thread 0 publishes the
  // point to evaluate through s_th
  double th[CB][3], lo[CB][3], hi[CB][3], rho[CB], J[CB];
  const double sc[3] = {c.dr, c.st0, c.st1};
#pragma unroll
  for (int b = 0; b < CB; ++b) {
#pragma unroll
    for (int q = 0; q < 3; ++q) th[b][q] = (b < nb) ? theta[(b0 + b) * 3 + q] : 0.0;
    int64_t ic[2];
    centre_of(c, th[b][1], th[b][2], ic);
    lo[b][0] = 0.0;
    hi[b][0] = (double)(c.N - 1) * c.dr;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      if (p < c.P) {
        // continuous fine index range of the coarse cell, kept 1e-6 inside
        const double ulo = (double)(ic[p] - c.R / 2) - 0.5 + 1e-6;
        const double uhi = (double)(ic[p] - c.R / 2 + c.R) - 0.5 - 1e-6;
        lo[b][1 + p] = ulo * sc[1 + p];
        hi[b][1 + p] = uhi * sc[1 + p];
      } else {
        lo[b][1 + p] = hi[b][1 + p] = 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) th[b][q] = fmin(fmax(th[b][q], lo[b][q]), hi[b][q]);
    rho[b] = 0.5;
  }
  auto publish = [&](const double (&pt)[CB][3]) {
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
      for (int b = 0; b < CB; ++b)
#pragma unroll
        for (int q = 0; q < 3; ++q) s_th[b][q] = pt[b][q];
    __syncthreads();
  };
  double out[CB][8], sv[CB][8];
  publish(th);
  eval_block<CB>(c, echo, s_th, nb, out, s_tap, red);
#pragma unroll
  for (int b = 0; b < CB; ++b) {
    finish(c, out[b], sv[b]);
    J[b] = sv[b][0] * sv[b][0] + sv[b][1] * sv[b][1];
  }
  for (int it = 0; it < iters; ++it) {
    double prop[CB][3];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      double g[3], gn = 0.0;
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        g[p] = (b < nb) ? 2.0 * (sv[b][0] * sv[b][2 + 2 * p] + sv[b][1] * sv[b][3 + 2 * p]) * sc[p]
                        : 0.0;
        gn += g[p] * g[p];
      }
      gn = sqrt(gn);
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const double z = (gn > 0.0) ? th[b][p] + rho[b] * g[p] / gn * sc[p] : th[b][p];
        prop[b][p] = fmin(fmax(z, lo[b][p]), hi[b][p]);
      }
    }
    double po[CB][8];
    publish(prop);
    eval_block<CB>(c, echo, s_th, nb, po, s_tap, red);
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      double ps[8];
      finish(c, po[b], ps);
      const double Jp = ps[0] * ps[0] + ps[1] * ps[1];
      if (b < nb && Jp >= J[b]) {
#pragma unroll
        for (int p = 0; p < 3; ++p) th[b][p] = prop[b][p];
#pragma unroll
        for (int q = 0; q < 8; ++q) sv[b][q] = ps[q];
        J[b] = Jp;
        rho[b] = fmin(2.0 * rho[b], 2.0);
      } else {
        rho[b] *= 0.5;
      }
    }
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      if (b < nb) {
#pragma unroll
        for (int q = 0; q < 3; ++q) theta[(b0 + b) * 3 + q] = th[b][q];
        if (Jout) Jout[b0 + b] = J[b];
      }
    }
  }
}

AdjCtx make_ctx(dsgrft_plan p) {
  AdjCtx c;
  c.M = p->M;
  c.N = p->N;
  c.P = p->P;
  c.R = p->R;
  c.K0 = p->K[0];
  c.K1 = p->K[1];
  c.ilo0 = p->ilo[0];
  c.ilo1 = p->ilo[1];
  c.dr = p->dr;
  c.prf = p->radar.prf;
  c.lam = p->lam;
  c.st0 = p->step[0];
  c.st1 = p->step[1];
  c.L = p->lat;
  return c;
}

}  // namespace

hipError_t launch_adjoint_forward(dsgrft_plan p, const float2 *echo,
                                  const double *theta, int B, double *J,
                                  double *saved, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_fwd<CB_FWD>, dim3((B + CB_FWD - 1) / CB_FWD), dim3(TPB), 0, s,
                     make_ctx(p),
                     echo, theta, B, J, saved);
  return hipGetLastError();
}

hipError_t launch_adjoint_backward(dsgrft_plan p, const float2 *echo,
                                   const double *theta, int B,
                                   const double *saved, const double *gJ,
                                   double *grad_theta, float2 *grad_echo,
                                   hipStream_t s) {
  (void)echo;
  if (grad_theta)
    hipLaunchKernelGGL(k_adj_theta, dim3((B + 255) / 256), dim3(256), 0, s, saved, gJ,
                       B, grad_theta);
  if (grad_echo) {
    const int slabs = (p->N + TPB * 8 - 1) / (TPB * 8);
    hipLaunchKernelGGL(k_adj_echo, dim3((unsigned)(p->M * slabs)), dim3(ECHO_TPB), 0, s,
                       make_ctx(p), theta, B, saved, gJ, grad_echo);
  }
  return hipGetLastError();
}

hipError_t launch_refine(dsgrft_plan p, const float2 *echo, double *theta, int B,
                         int iters, double *J, hipStream_t s) {
  hipLaunchKernelGGL(k_refine<CB_REF>, dim3((B + CB_REF - 1) / CB_REF), dim3(TPB), 0, s,
                     make_ctx(p),
                     echo, theta, B, iters, J);
  return hipGetLastError();
}
