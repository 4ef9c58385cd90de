// Stages a5 + a6: LRT detection on the reduced map and peak parameters.
//
// Threshold test of Sec. III-C (eqs. (31), (33)) and Alg. 3: every reduced
// map entry (cell, row) with power above gamma^2 is a detection carrying its
// best fine cell; parameters follow eq. (72) with kappa = 1 in FP64:
// r0 = n0 dr, (v, a, j) = (coarse centre + fine offset) * fine step.
//
// The same kernels run a cell-averaging CFAR along range instead of the
// fixed threshold (not in the paper): entry (cell, r) is a detection when its
// power exceeds alpha times the mean of rows r' of the same cell with
// guard < |r' - r| <= guard + train inside the map, the mean a float64 sum
// in increasing r' divided by the number of those rows (no rows: no
// detection).
//
// Deterministic ordered compaction in three kernels: per-chunk counts and
// chunk maxima, one exclusive scan (and the global maximum, smallest flat
// index on ties), then an ordered write per chunk.  A chunk is 4096 map
// entries; thread t of a chunk owns entries t, t + 256, ... .
#include <mutex>

#include "internal.h"

namespace {

constexpr int CHUNK = 4096, TPB = 256, PER = CHUNK / TPB;

struct Best {
  float v;
  int64_t i;
};

__device__ inline bool better(float v, int64_t i, float bv, int64_t bi) {
  return v > bv || (v == bv && i < bi);
}

// Detection tests on entry i of a reduced map.
//
// LRT (eq. (33)): power > gamma^2 = -M sigma^2 ln P_FA, formed in FP64 in
// the order (-M sigma^2) ln P_FA; ln P_FA comes from the host (one value per
// call), sigma^2 from the host or, when s2p is set, from device memory (an
// estimate written earlier on the same stream).
struct LrtTest {
  double neg_m, s2, ln_pfa;
  const double *s2p;
  __device__ bool operator()(const float *__restrict__ pm, int64_t i) const {
    const double sigma2 = s2p != nullptr ? *s2p : s2;
    return (double)pm[i] > (neg_m * sigma2) * ln_pfa;
  }
};

struct CfarTest {
  int rows, guard, train;
  double alpha;
  __device__ bool operator()(const float *__restrict__ pm, int64_t i) const {
    const int64_t base = i - i % rows;
    const int r = (int)(i - base);
    const int lo = r - guard - train, hi = r + guard + train;
    double sum = 0.0;
    int cnt = 0;
    for (int q = (lo > 0 ? lo : 0); q < r - guard; ++q) {
      sum += (double)pm[base + q];
      ++cnt;
    }
    for (int q = r + guard + 1; q <= hi && q < rows; ++q) {
      sum += (double)pm[base + q];
      ++cnt;
    }
    return cnt > 0 && (double)pm[i] > alpha * (sum / (double)cnt);
  }
};

template <class Test>
__global__ __launch_bounds__(TPB) void k_det_count(const float *__restrict__ pm,
                                                   int64_t total, Test test,
                                                   int32_t *__restrict__ counts,
                                                   float *__restrict__ bv_out,
                                                   int64_t *__restrict__ bi_out) {
  __shared__ int s_cnt[TPB / 64];
  __shared__ float s_v[TPB];
  __shared__ int64_t s_i[TPB];
  const int64_t base = (int64_t)blockIdx.x * CHUNK;
  const int tid = threadIdx.x;
  int cnt = 0;
  float bv = -INFINITY;
  int64_t bi = INT64_MAX;
  for (int j = 0; j < PER; ++j) {
    const int64_t i = base + tid + (int64_t)TPB * j;
    if (i < total) {
      const float v = pm[i];
      cnt += test(pm, i) ? 1 : 0;
      if (better(v, i, bv, bi)) {
        bv = v;
        bi = i;
      }
    }
  }
  for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o);
  if ((tid & 63) == 0) s_cnt[tid >> 6] = cnt;
  s_v[tid] = bv;
  s_i[tid] = bi;
  __syncthreads();
  for (int s = TPB / 2; s >= 1; s >>= 1) {
    if (tid < s && better(s_v[tid + s], s_i[tid + s], s_v[tid], s_i[tid])) {
      s_v[tid] = s_v[tid + s];
      s_i[tid] = s_i[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0) {
    int c = 0;
    for (int w = 0; w < TPB / 64; ++w) c += s_cnt[w];
    counts[blockIdx.x] = c;
    bv_out[blockIdx.x] = s_v[0];
    bi_out[blockIdx.x] = s_i[0];
  }
}

struct PeakCtx {
  const int64_t *cells;
  int64_t cc_begin;
  int rows, n_begin, R, P, K0, K1, K2, i0, i1, i2, S0;
  double dr, st0, st1, st2;
};

__device__ inline dsgrft_peak make_peak(const PeakCtx &c, int64_t flat, float pw,
                                        int32_t f) {
  dsgrft_peak pk;
  const int64_t pos = flat / c.rows;
  const int r = (int)(flat % c.rows);
  const int64_t k = cell_id(c.cells, c.cc_begin, pos);
  int Ks[3] = {c.K0, c.K1, c.K2}, il[3] = {c.i0, c.i1, c.i2};
  int64_t ic[3], fo[3];
  coarse_centre(Ks, il, c.R, c.P, k, ic, c.S0);
  fine_offsets(c.R, c.P, f, fo, c.S0);
  pk.coarse = k;
  pk.row = c.n_begin + r;
  pk.fine = f;
  pk.power = pw;
  pk.pad_ = 0.f;
  pk.r0 = (double)(c.n_begin + r) * c.dr;
  pk.v = (double)(ic[0] + fo[0]) * c.st0;
  pk.a = (double)(ic[1] + fo[1]) * c.st1;
  pk.j = (double)(ic[2] + fo[2]) * c.st2;
  return pk;
}

// Single workgroup: exclusive scan of the chunk counts in place, total count,
// and the global maximum.
__global__ __launch_bounds__(TPB) void k_det_scan(
    int32_t *__restrict__ counts, const float *__restrict__ bv,
    const int64_t *__restrict__ bi, int64_t nchunks, const float *__restrict__ pm,
    const int32_t *__restrict__ argf, PeakCtx ctx, int32_t *__restrict__ total,
    dsgrft_peak *__restrict__ best) {
  __shared__ int s_sum[TPB];
  __shared__ float s_v[TPB];
  __shared__ int64_t s_i[TPB];
  const int tid = threadIdx.x;
  const int64_t per = (nchunks + TPB - 1) / TPB;
  const int64_t lo = tid * per, hi = (lo + per < nchunks) ? lo + per : nchunks;
  int sum = 0;
  float v = -INFINITY;
  int64_t idx = INT64_MAX;
  for (int64_t c = lo; c < hi; ++c) {
    sum += counts[c];
    if (better(bv[c], bi[c], v, idx)) {
      v = bv[c];
      idx = bi[c];
    }
  }
  s_sum[tid] = sum;
  s_v[tid] = v;
  s_i[tid] = idx;
  __syncthreads();
  if (tid == 0) {  // serial scan of 256 partial sums
    int run = 0;
    for (int t = 0; t < TPB; ++t) {
      int x = s_sum[t];
      s_sum[t] = run;
      run += x;
    }
    *total = run;
  }
  __syncthreads();
  int run = s_sum[tid];
  for (int64_t c = lo; c < hi; ++c) {
    int x = counts[c];
    counts[c] = run;
    run += x;
  }
  for (int s = TPB / 2; s >= 1; s >>= 1) {
    if (tid < s && better(s_v[tid + s], s_i[tid + s], s_v[tid], s_i[tid])) {
      s_v[tid] = s_v[tid + s];
      s_i[tid] = s_i[tid + s];
    }
    __syncthreads();
  }
  if (tid == 0 && best != nullptr) {
    const int64_t fl = s_i[0];
    if (fl == INT64_MAX) {  // no comparable entry (all NaN)
      dsgrft_peak z = {};
      z.coarse = -1;
      z.power = NAN;
      *best = z;
    } else {
      *best = make_peak(ctx, fl, pm[fl], argf[fl]);
    }
  }
}

template <class Test>
__global__ __launch_bounds__(TPB) void k_det_write(
    const float *__restrict__ pm, const int32_t *__restrict__ argf,
    int64_t total, Test test, const int32_t *__restrict__ offsets,
    PeakCtx ctx, dsgrft_peak *__restrict__ peaks, int32_t cap) {
  __shared__ int s_w[TPB / 64];
  const int64_t base = (int64_t)blockIdx.x * CHUNK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int run = offsets[blockIdx.x];
  for (int j = 0; j < PER; ++j) {
    const int64_t i = base + tid + (int64_t)TPB * j;
    const bool hit = (i < total) && test(pm, i);
    const unsigned long long mask = __ballot(hit);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) s_w[wave] = __popcll(mask);
    __syncthreads();
    int wofs = 0, tot = 0;
    for (int w = 0; w < TPB / 64; ++w) {
      if (w < wave) wofs += s_w[w];
      tot += s_w[w];
    }
    if (hit) {
      const int pos = run + wofs + before;
      if (pos < cap) peaks[pos] = make_peak(ctx, i, pm[i], argf[i]);
    }
    run += tot;
    __syncthreads();
  }
}

__global__ __launch_bounds__(TPB) void k_noise_partial(const float2 *__restrict__ e,
                                                       int64_t n,
                                                       double *__restrict__ part) {
  __shared__ double s[TPB];
  const int64_t base = (int64_t)blockIdx.x * 65536;
  double acc = 0.0;
  for (int j = threadIdx.x; j < 65536; j += TPB) {
    const int64_t i = base + j;
    if (i < n) {
      const float2 v = e[i];
      acc += (double)v.x * v.x + (double)v.y * v.y;
    }
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int st = TPB / 2; st >= 1; st >>= 1) {
    if (threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void k_noise_final(const double *__restrict__ part, int64_t nb, int64_t n,
                              double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double acc = 0.0;
  for (int64_t i = 0; i < nb; ++i) acc += part[i];
  *out = acc / (double)n;
}

}  // namespace

namespace {

template <class Test>
hipError_t launch_detect_t(dsgrft_plan p, const float *pmax, const int32_t *argf,
                           const int64_t *cells, int64_t cc_begin, int64_t n, Test test,
                           dsgrft_peak *peaks, int32_t cap, int32_t *count,
                           dsgrft_peak *best, hipStream_t s) {
  const int64_t total = n * p->rows;
  const int64_t nch = (total + CHUNK - 1) / CHUNK;
  char *ws = (char *)p->det_ws;
  int32_t *counts = (int32_t *)ws;
  float *bv = (float *)(ws + 8 * ((nch * 4 + 7) / 8));
  int64_t *bi = (int64_t *)((char *)bv + 8 * ((nch * 4 + 7) / 8));
  PeakCtx ctx{cells, cc_begin, p->rows, p->n_begin, p->R, p->P, p->K[0], p->K[1],
              p->K[2], p->ilo[0], p->ilo[1], p->ilo[2], p->S0, p->dr,
              p->step[0], p->step[1], p->step[2]};
  hipLaunchKernelGGL(k_det_count<Test>, dim3((unsigned)nch), dim3(TPB), 0, s, pmax, total,
                     test, counts, bv, bi);
  hipLaunchKernelGGL(k_det_scan, dim3(1), dim3(TPB), 0, s, counts, bv, bi, nch, pmax,
                     argf, ctx, count, best);
  hipLaunchKernelGGL(k_det_write<Test>, dim3((unsigned)nch), dim3(TPB), 0, s, pmax, argf,
                     total, test, counts, ctx, peaks, cap);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_detect(dsgrft_plan p, const float *pmax, const int32_t *argf,
                         const int64_t *cells, int64_t cc_begin, int64_t n,
                         double sigma2, const double *d_sigma2, double ln_pfa,
                         dsgrft_peak *peaks, int32_t cap, int32_t *count,
                         dsgrft_peak *best, hipStream_t s) {
  const LrtTest test{-(double)p->M, sigma2, ln_pfa, d_sigma2};
  return launch_detect_t(p, pmax, argf, cells, cc_begin, n, test, peaks, cap, count, best,
                         s);
}

hipError_t launch_detect_cfar(dsgrft_plan p, const float *pmax, const int32_t *argf,
                              const int64_t *cells, int64_t cc_begin, int64_t n, int guard,
                              int train, double alpha, dsgrft_peak *peaks, int32_t cap,
                              int32_t *count, dsgrft_peak *best, hipStream_t s) {
  return launch_detect_t(p, pmax, argf, cells, cc_begin, n,
                         CfarTest{p->rows, guard, train, alpha}, peaks, cap, count, best, s);
}

size_t detect_ws_bytes(int64_t max_entries) {
  const int64_t nch = (max_entries + CHUNK - 1) / CHUNK;
  return (size_t)(2 * 8 * ((nch * 4 + 7) / 8) + 8 * nch + 64);
}

hipError_t launch_noise_power(dsgrft_plan p, const float2 *echo, double *out,
                              hipStream_t s) {
  const int64_t n = (int64_t)p->M * p->N;
  const int64_t nb = (n + 65535) / 65536;
  double *part = p->adj_ws;
  hipLaunchKernelGGL(k_noise_partial, dim3((unsigned)nb), dim3(TPB), 0, s, echo, n,
                     part);
  hipLaunchKernelGGL(k_noise_final, dim3(1), dim3(64), 0, s, part, nb, n, out);
  return hipGetLastError();
}

// ---- plan-free noise power that allocates nothing --------------------------
//
// The partial sums of dsgrft_noise_power_noalloc live in `scratch`, a static
// device array of DSGRFT_NOALLOC_MAX_PARTS doubles (one per 65536 echo
// samples; each GPU holds its own copy until the process ends).  Host code
// must not pass `scratch` itself to a kernel (on the host it names a
// host-side stand-in): the device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and cached.  The partial
// kernel writes every entry the final kernel reads, so nothing needs
// clearing between calls; calls that overlap on one GPU race on the array.
static __device__ __align__(256) double scratch[DSGRFT_NOALLOC_MAX_PARTS];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_for_device(int dev, double **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double *)ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" dsgrft_status dsgrft_noise_power_noalloc(const void *d_echo, int32_t M, int32_t N,
                                                    double *d_sigma2, void *stream) {
  if (!d_echo || !d_sigma2 || M < 1 || N < 1) return DSGRFT_E_INVALID;
  const int64_t n = (int64_t)M * N;
  const int64_t nb = (n + 65535) / 65536;
  if (nb > DSGRFT_NOALLOC_MAX_PARTS) return DSGRFT_E_INVALID;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return DSGRFT_E_DEVICE;
  if (dev < 0 || dev >= kMaxDevices) return DSGRFT_E_UNSUPPORTED;
  double *part = nullptr;
  if (scratch_for_device(dev, &part) != hipSuccess) return DSGRFT_E_DEVICE;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_noise_partial, dim3((unsigned)nb), dim3(TPB), 0, s,
                     (const float2 *)d_echo, n, part);
  hipLaunchKernelGGL(k_noise_final, dim3(1), dim3(64), 0, s, part, nb, n, d_sigma2);
  return hipGetLastError() == hipSuccess ? DSGRFT_OK : DSGRFT_E_DEVICE;
}
