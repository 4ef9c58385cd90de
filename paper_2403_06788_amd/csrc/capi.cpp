// C ABI of the DS-GRFT library: plan construction (lattice derivation,
// validation, workspace sizing, fine tables) and the stream-ordered entry
// points that sequence the kernels.  See include/dsgrft.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

namespace {

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Nearest integer when x lies within tol of it; sets ok accordingly.
long long snap(double x, double tol, bool &ok) {
  double r = std::nearbyint(x);
  ok = std::fabs(x - r) <= tol;
  return (long long)r;
}

// Outward-rounded index bounds of [lo, hi] on the lattice i * step; a bound
// within 1e-6 of a lattice point counts as on it.
void index_bounds(double lo, double hi, double step, long long &il, long long &ih) {
  bool ok;
  double xl = lo / step, xh = hi / step;
  long long s = snap(xl, 1e-6, ok);
  il = ok ? s : (long long)std::floor(xl);
  s = snap(xh, 1e-6, ok);
  ih = ok ? s : (long long)std::ceil(xh);
}

template <typename T>
hipError_t dalloc(T **p, size_t bytes, size_t &total) {
  *p = nullptr;
  if (bytes == 0) return hipSuccess;
  hipError_t e = hipMalloc((void **)p, bytes);
  if (e == hipSuccess) total += bytes;
  return e;
}

void release(dsgrft_plan p) {
  if (!p) return;
  void *bufs[] = {p->F32, p->F16, p->FBF16, p->F8, p->FS16, p->FSB16, p->FS8, p->sym_cols, p->u_off, p->u_psi,
                  p->Gbuf[0], p->gscbuf[0], p->fft_tw, p->fd_tw, p->fd_spec, p->fd_E,
                  p->kt_spec, p->kt_invd, p->packed, p->det_ws, p->adj_ws, p->g_shift};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  hipEvent_t evs[] = {p->ev_start, p->ev_g[0], p->ev_g[1], p->ev_f[0], p->ev_f[1]};
  for (hipEvent_t e : evs)
    if (e) (void)hipEventDestroy(e);
  if (p->aux) (void)hipStreamDestroy(p->aux);
  delete p;
}

bool on_plan_device(dsgrft_plan p) {
  int d = -1;
  return hipGetDevice(&d) == hipSuccess && d == p->device;
}

dsgrft_status check_form(dsgrft_plan p, dsgrft_form form, int split) {
  if (p->kt && form != DSGRFT_FORM_F32_FFT)
    return (form >= DSGRFT_FORM_F32 && form <= DSGRFT_FORM_FP8_SYM) ? DSGRFT_E_UNSUPPORTED
                                                                   : DSGRFT_E_INVALID;
  switch (form) {
    case DSGRFT_FORM_F32:
      return split == 1 ? DSGRFT_OK : DSGRFT_E_INVALID;
    case DSGRFT_FORM_F32_FFT:
      if (split != 1) return DSGRFT_E_INVALID;
      return p->fft_tw ? DSGRFT_OK : DSGRFT_E_UNSUPPORTED;
    case DSGRFT_FORM_F16_3M:
    case DSGRFT_FORM_F16_SYM:
      return split == 1 ? DSGRFT_OK : DSGRFT_E_INVALID;
    case DSGRFT_FORM_BF16_GLO:
      return split == 2 ? DSGRFT_OK : DSGRFT_E_INVALID;
    case DSGRFT_FORM_BF16_SYM:
      return (split == 2 || split == 3) ? DSGRFT_OK : DSGRFT_E_INVALID;
    case DSGRFT_FORM_FP8_SYM:
      if (split != 3 && split != 4) return DSGRFT_E_INVALID;
      return p->FS8 ? DSGRFT_OK : DSGRFT_E_UNSUPPORTED;
    case DSGRFT_FORM_F16:
    case DSGRFT_FORM_BF16:
    case DSGRFT_FORM_FP8:
      return (split >= 1 && split <= 4) ? DSGRFT_OK : DSGRFT_E_INVALID;
    default:
      return DSGRFT_E_INVALID;
  }
}

// Bytes written per gathered sample: complex64, or 2 / 4 planes (lo parts
// of G from split 3 on, and in BF16_GLO) of 2-byte or 1-byte components.
double gather_bytes(dsgrft_form form, int split) {
  if (form == DSGRFT_FORM_F32 || form == DSGRFT_FORM_F32_FFT) return 8.0;
  const double planes =
      (split >= 3 || form == DSGRFT_FORM_BF16_GLO || form == DSGRFT_FORM_BF16_SYM) ? 4.0 : 2.0;
  return planes * ((form == DSGRFT_FORM_FP8 || form == DSGRFT_FORM_FP8_SYM) ? 1.0 : 2.0);
}

// Executed MFMA flops per gathered unit of a fine-search launch: padded rows
// x table columns x padded pulses x 2 x real products per (row, column,
// pulse); 0 for the vector-ALU forms.
double mfma_flops_per_unit(dsgrft_plan p, dsgrft_form form, int split) {
  double prod, cols = (double)p->Cp;
  switch (form) {
    case DSGRFT_FORM_F16:
    case DSGRFT_FORM_BF16:
    case DSGRFT_FORM_FP8: prod = 4.0 * split; break;
    case DSGRFT_FORM_BF16_GLO: prod = 8.0; break;
    case DSGRFT_FORM_F16_3M: prod = 3.0; break;
    case DSGRFT_FORM_F16_SYM: prod = 4.0; cols = 32.0 * p->FBs; break;
    case DSGRFT_FORM_BF16_SYM:
    case DSGRFT_FORM_FP8_SYM: prod = 4.0 * split; cols = 32.0 * p->FBs; break;
    default: return 0.0;
  }
  return (double)p->rows_p * cols * (double)p->Mp * 2.0 * prod;
}

// Stages a0..a4 over n listed cells, batch by batch.  pmax/argf may be NULL
// (full-map only), full may be NULL.
//
// Two-stream pipeline: the producer stream `aux` runs the per-echo transforms
// and, per batch of gathered units, the unit tables, the coarse compensation
// and the gather into slot b % 2 of the gathered buffer; the caller's stream
// runs the fine search of batch b on that slot and the reductions.  Events
// order the slots (the fine search of b waits for its gather; the gather of
// b + 2 waits until the fine search of b has read the slot), so the
// memory-bound producer work of batch b + 1 overlaps the compute-bound fine
// search of batch b.  `aux` first waits for everything already enqueued on
// the caller's stream, and the caller's stream waits for every gather, so
// the call stays ordered on the caller's stream as a whole.
dsgrft_status run_search(dsgrft_plan p, dsgrft_form form, int split,
                         const float2 *echo, const int64_t *cells,
                         int64_t cc_begin, int64_t n, float *pmax, int32_t *argf,
                         float *full, hipStream_t s) {
  const int64_t Bc = p->batch_cells, Bu = p->batch_units;
  hipStream_t sa = p->aux;
  DS_TRY(hipEventRecord(p->ev_start, s));
  DS_TRY(hipStreamWaitEvent(sa, p->ev_start, 0));
  if (p->fd) DS_TRY(launch_range_fft(p, echo, sa));
  if (p->kt) DS_TRY(launch_keystone(p, sa));
  if (fp16_form(form)) DS_TRY(launch_echo_shift(p, echo, sa));
  const GatherSrc src = gather_src(p, echo);
  int64_t b = 0;
  for (int64_t c0 = 0; c0 < n; c0 += Bc) {
    const int64_t nc = (n - c0) < Bc ? (n - c0) : Bc;
    DS_TRY(launch_fill_u64(p->packed, nc * p->rows, s));
    const int64_t nut = nc * p->R3;
    const int64_t *cl = cells ? cells + c0 : nullptr;
    float *fl = full ? full + c0 * p->rows * p->n_fine : nullptr;
    for (int64_t u0 = 0; u0 < nut; u0 += Bu, ++b) {
      const int64_t nu = (nut - u0) < Bu ? (nut - u0) : Bu;
      const int slot = (int)(b & 1);
      p->G = p->Gbuf[slot];
      p->g_scale = p->gscbuf[slot];
      if (b >= 2) DS_TRY(hipStreamWaitEvent(sa, p->ev_f[slot], 0));
      DS_TRY(launch_unit_tables(p, cl, cc_begin + c0, u0, nu, sa));
      if (p->kt)
        DS_TRY(launch_kt_shift(p, cl, cc_begin + c0, u0, nu, sa));
      else if (p->fd)
        DS_TRY(launch_fd_shift(p, cl, cc_begin + c0, u0, nu, p->R3, sa));
      auto &pr = p->prof;
      const bool tg = pr.ng < pr.cap, tf = pr.nf < pr.cap;
      const double samples = (double)nu * p->rows * p->M;
      const double bg = gather_bytes(form, split);
      if (tg) DS_TRY(hipEventRecord(pr.ev_g[2 * pr.ng], sa));
      if (form == DSGRFT_FORM_F32 || form == DSGRFT_FORM_F32_FFT)
        DS_TRY(launch_gather_f32(p, src, nu, sa));
      else
        DS_TRY(launch_gather_lp(p, form, split, src, nu, sa));
      if (tg) {
        DS_TRY(hipEventRecord(pr.ev_g[2 * pr.ng + 1], sa));
        pr.ng++;
        pr.gbytes += samples * (8.0 + bg);
      }
      DS_TRY(hipEventRecord(p->ev_g[slot], sa));
      DS_TRY(hipStreamWaitEvent(s, p->ev_g[slot], 0));
      if (tf) DS_TRY(hipEventRecord(pr.ev_f[2 * pr.nf], s));
      if (form == DSGRFT_FORM_F32)
        DS_TRY(launch_fine_f32(p, nu, u0, fl, 0, s));
      else if (form == DSGRFT_FORM_F32_FFT)
        DS_TRY(launch_fine_fft(p, nu, u0, fl, s));
      else
        DS_TRY(launch_fine_mfma(p, form, split, nu, u0, fl, s));
      if (tf) {
        DS_TRY(hipEventRecord(pr.ev_f[2 * pr.nf + 1], s));
        pr.nf++;
        pr.fcp += samples * p->C;
        pr.fflops += 8.0 * samples * p->C;
        pr.fxflops += (double)nu * mfma_flops_per_unit(p, form, split);
      }
      DS_TRY(hipEventRecord(p->ev_f[slot], s));
    }
    if (pmax && argf)
      DS_TRY(launch_unpack(p, nc, pmax + c0 * p->rows, argf + c0 * p->rows, s));
  }
  return DSGRFT_OK;
}

}  // namespace

// Zero-padded range-FFT length of the frequency-domain mGIFT: the smallest
// power of two >= N + W, W = ceil(sum_p max|i_c,p| (M-1)^p M^(3-p) / (R M^3))
// + 1 bounds every coarse walk in bins.
// Columns of the conjugate-pair table: fine cell f (offsets f % R - R/2 and
// f / R - R/2, or f - R/2 for P = 1) and the cell with the negated offsets,
// once per pair, the smaller index first; cells whose negated offsets leave
// the lattice (an offset of -R/2 for even R) and the centre stand alone.
void sym_columns(int R, int P, int C, std::vector<int32_t> &plus,
                 std::vector<int32_t> &minus) {
  const int h = R / 2;
  for (int f = 0; f < C; ++f) {
    const int o1 = (P >= 2 ? f % R : f) - h, o2 = P >= 2 ? f / R - h : 0;
    const int n1 = h - o1, n2 = h - o2;
    int g = -1;
    if (n1 >= 0 && n1 < R && (P < 2 || (n2 >= 0 && n2 < R))) g = P >= 2 ? n1 + R * n2 : n1;
    if (g >= 0 && g < f) continue;  // listed with g
    plus.push_back(f);
    minus.push_back(g > f ? g : -1);
  }
}

int fd_pad_length(dsgrft_plan p) {
  const __int128 M = p->M;
  __int128 tot = 0;
  for (int q = 0; q < p->P; ++q) {
    const long long lo = (long long)p->ilo[q] + p->h;
    const long long hi = (long long)p->ilo[q] + (long long)(p->K[q] - 1) * p->R + p->h;
    const long long mag = (lo < 0 ? -lo : lo) > (hi < 0 ? -hi : hi) ? (lo < 0 ? -lo : lo)
                                                                     : (hi < 0 ? -hi : hi);
    __int128 t = mag;
    for (int e = 0; e <= q; ++e) t *= (M - 1);
    for (int e = 0; e < 2 - q; ++e) t *= M;
    tot += t;
  }
  const __int128 den = (__int128)p->R * M * M * M;
  const long long W = (long long)((tot + den - 1) / den) + 1;
  long long need = (long long)p->N + W, L = 1;
  while (L < need && L <= (1LL << 40)) L *= 2;
  return L > (1LL << 30) ? (1 << 30) : (int)L;
}

extern "C" {

const char *dsgrft_status_string(dsgrft_status s) {
  switch (s) {
    case DSGRFT_OK: return "ok";
    case DSGRFT_E_INVALID: return "invalid argument";
    case DSGRFT_E_NOMEM: return "out of device memory";
    case DSGRFT_E_DEVICE: return "HIP runtime error";
    case DSGRFT_E_UNSUPPORTED: return "unsupported request";
    case DSGRFT_E_CAPACITY: return "output capacity exceeded";
    default: return "unknown status";
  }
}

dsgrft_status dsgrft_plan_create(const dsgrft_radar *radar,
                                 const dsgrft_config *cfg, dsgrft_plan *out) {
  if (!radar || !cfg || !out) return DSGRFT_E_INVALID;
  *out = nullptr;
  if (!finite_pos(radar->fc) || !finite_pos(radar->fs) ||
      !finite_pos(radar->prf) || !finite_pos(radar->c))
    return DSGRFT_E_INVALID;
  if (!std::isfinite(radar->kappa)) return DSGRFT_E_INVALID;
  if (radar->kappa != 1.0) return DSGRFT_E_UNSUPPORTED;
  const int M = cfg->M, N = cfg->N, P = cfg->order;
  if (M < 1 || N < 1 || P < 1 || P > 3 || cfg->batch < 0) return DSGRFT_E_INVALID;
  if (cfg->mgift < 0 || cfg->mgift > 2) return DSGRFT_E_INVALID;
  if (M > (1 << 20) || N > (1 << 28)) return DSGRFT_E_INVALID;
  int nb = cfg->n_begin, ne = cfg->n_end;
  if (nb == 0 && ne == 0) ne = N;
  if (nb < 0 || nb >= ne || ne > N) return DSGRFT_E_INVALID;
  const double ratio = radar->fc / radar->fs;
  bool ok;
  const long long R = snap(ratio, 1e-9 * (ratio > 1.0 ? ratio : 1.0), ok);
  if (!ok || R < 1 || R > 4096) return DSGRFT_E_INVALID;

  dsgrft_plan p = new (std::nothrow) dsgrft_plan_s();
  if (!p) return DSGRFT_E_NOMEM;
  p->radar = *radar;
  p->cfg = *cfg;
  p->M = M;
  p->N = N;
  p->P = P;
  p->n_begin = nb;
  p->n_end = ne;
  p->rows = ne - nb;
  p->R = (int)R;
  p->h = (int)(R / 2);
  p->lam = radar->c / radar->fc;
  p->dr = radar->c / (2.0 * radar->fs);
  p->T = M / radar->prf;
  p->step[0] = p->lam / (2.0 * p->T);
  p->step[1] = p->lam / (p->T * p->T);
  p->step[2] = 3.0 * p->lam / (p->T * p->T * p->T);
  // lattice per order
  __int128 bound = 0;
  const __int128 M3 = (__int128)M * M * M;
  for (int q = 0; q < 3; ++q) {
    if (q < P) {
      const dsgrft_axis &ax = cfg->axis[q];
      if (!std::isfinite(ax.min) || !std::isfinite(ax.max) || ax.min > ax.max) {
        delete p;
        return DSGRFT_E_INVALID;
      }
      const double xl = ax.min / p->step[q], xh = ax.max / p->step[q];
      if (std::fabs(xl) > 1e15 || std::fabs(xh) > 1e15) {
        delete p;
        return DSGRFT_E_INVALID;
      }
      long long il, ih;
      index_bounds(ax.min, ax.max, p->step[q], il, ih);
      const long long Kq = (ih - il + 1 + R - 1) / R;
      const long long top = il + Kq * R;
      if (il < -(1LL << 30) || top > (1LL << 30) || Kq > (1LL << 30)) {
        delete p;
        return DSGRFT_E_INVALID;
      }
      p->ilo[q] = (int)il;
      p->K[q] = (int)Kq;
      const long long mag = (il < 0 ? -il : il) > (top < 0 ? -top : top)
                                ? (il < 0 ? -il : il)
                                : (top < 0 ? -top : top);
      bound += (__int128)mag * M3;
    } else {
      p->ilo[q] = 0;
      p->K[q] = 1;
    }
  }
  if (2 * bound + (__int128)R * M3 >= ((__int128)1 << 62)) {
    delete p;
    return DSGRFT_E_INVALID;
  }
  p->lat.M = M;
  p->lat.M3 = (int64_t)M3;
  p->lat.RM3 = (int64_t)(R * M3);
  p->S0 = (int)R;
  p->gK0 = p->K[0];
  p->gilo0 = p->ilo[0];
  p->fd = cfg->mgift != 0;
  p->kt = cfg->mgift == 2;
  if (p->fd) {
    p->fd_np = fd_pad_length(p);  // from the DS-GRFT lattice in both modes
    if (p->fd_np > 16384) {
      delete p;
      return DSGRFT_E_UNSUPPORTED;
    }
  }
  long long nf = 1, C = 1;
  for (int q = 0; q < P; ++q) nf *= R;
  for (int q = 0; q < (P < 2 ? P : 2); ++q) C *= R;
  if (p->kt) {
    // DS-KT-MFP lattice (velocity folding, eq. (23)): fine velocity index
    // i1 = q M + i1', i1' in [-M/2, M/2); the folding factors cover the
    // axis's indices [i_lo, i_lo + K1 R), the acceleration axis keeps the
    // DS-GRFT coarse cells, and the fine space is M x R.
    if (P != 2 || !fft_form_supported(M)) {
      delete p;
      return DSGRFT_E_UNSUPPORTED;
    }
    const long long i_lo = p->ilo[0], i_hi = i_lo + (long long)p->K[0] * R - 1;
    const long long q_lo = (long long)floor_div(i_lo + M / 2, M);
    const long long q_hi = (long long)floor_div(i_hi + M / 2, M);
    const long long lo0 = q_lo * M - M / 2, top0 = (q_hi + 1) * M - M / 2;
    const long long mag0 = (lo0 < 0 ? -lo0 : lo0) > (top0 < 0 ? -top0 : top0)
                               ? (lo0 < 0 ? -lo0 : lo0) : (top0 < 0 ? -top0 : top0);
    const long long il1 = p->ilo[1], top1 = il1 + (long long)p->K[1] * R;
    const long long mag1 = (il1 < 0 ? -il1 : il1) > (top1 < 0 ? -top1 : top1)
                               ? (il1 < 0 ? -il1 : il1) : (top1 < 0 ? -top1 : top1);
    if (lo0 < -(1LL << 30) || top0 > (1LL << 30) ||
        2 * ((__int128)mag0 + mag1) * M3 + (__int128)R * M3 >= ((__int128)1 << 62)) {
      delete p;
      return DSGRFT_E_INVALID;
    }
    p->kt_q_lo = (int)q_lo;
    p->kt_na = (int)(q_hi - q_lo + 1);
    p->K[0] = p->kt_na;
    p->ilo[0] = (int)lo0;
    p->S0 = M;
    nf = (long long)M * R;
    C = nf;
  }
  p->n_coarse = (int64_t)p->K[0] * p->K[1] * p->K[2];
  if (nf >= 0xffffffffLL) {
    delete p;
    return DSGRFT_E_INVALID;
  }
  p->n_fine = nf;
  p->C = (int)C;
  p->R3 = (P == 3) ? (int)R : 1;
  // padded sizes
  p->Mp = (M + KTILE - 1) / KTILE * KTILE;
  p->rows_p = (p->rows + ROWTILE - 1) / ROWTILE * ROWTILE;
  p->Cp = (p->C + COLTILE - 1) / COLTILE * COLTILE;
  p->KB = p->Mp / 16;
  p->NB = p->rows_p / 32;
  p->FB = p->Cp / 32;
  // batching: gathered units of at most ~512 MiB at 8 bytes per sample
  const size_t per_unit = (size_t)p->rows_p * p->Mp * 8;
  const int64_t total_units = p->n_coarse * p->R3;
  int64_t bu = cfg->batch > 0 ? cfg->batch : (int64_t)((512ull << 20) / per_unit);
  if (bu < 1) bu = 1;
  if (bu > total_units) bu = total_units;
  if (p->R3 > 1) {
    if (bu >= p->R3) {
      p->batch_cells = bu / p->R3;
      bu = p->batch_cells * p->R3;
    } else {
      p->batch_cells = 1;
    }
  } else {
    p->batch_cells = bu;
  }
  p->batch_units = bu;

  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return DSGRFT_E_DEVICE;
  }
  size_t tot = 0;
  // the GEMM-form fine tables are not built for DS-KT-MFP (FFT form only)
  const size_t f16b = p->kt ? 0 : (size_t)4 * p->Cp * p->Mp * 2;
  std::vector<int32_t> sym_plus, sym_minus;
  if (!p->kt) sym_columns(p->R, p->P, p->C, sym_plus, sym_minus);
  p->FBs = (int)((sym_plus.size() + 63) / 64 * 2);
  const size_t sym_cols_n = (size_t)p->FBs * 32;
  p->det_ws_bytes = detect_ws_bytes(p->n_coarse * (int64_t)p->rows);
  const int64_t noise_parts = ((int64_t)M * N + 65535) / 65536;
  p->adj_ws_bytes = (size_t)(noise_parts + 64) * sizeof(double);
  if (dalloc(&p->F32, f16b ? (size_t)p->Mp * p->Cp * sizeof(float2) : 0, tot) != hipSuccess ||
      dalloc(&p->F16, f16b, tot) != hipSuccess ||
      dalloc(&p->FBF16, f16b, tot) != hipSuccess ||
      dalloc(&p->F8, f16b ? (size_t)4 * p->Cp * p->Mp : 0, tot) != hipSuccess ||
      dalloc(&p->FS16, (size_t)2 * p->FBs * p->KB * 64 * sizeof(uint4), tot) != hipSuccess ||
      dalloc(&p->FSB16, (size_t)4 * p->FBs * p->KB * 64 * sizeof(uint4), tot) != hipSuccess ||
      dalloc(&p->FS8, f16b ? (size_t)2 * p->FBs * p->KB * 64 * sizeof(uint4) : 0, tot) !=
          hipSuccess ||
      dalloc(&p->sym_cols, 2 * sym_cols_n * sizeof(int32_t), tot) != hipSuccess ||
      dalloc(&p->gscbuf[0], 2 * (size_t)bu * p->rows_p * sizeof(int32_t), tot) != hipSuccess ||
      (fft_form_supported(M) &&
       dalloc(&p->fft_tw, fft_table_elems(M, p->R, P) * sizeof(float2), tot) != hipSuccess) ||
      (p->fd &&
       (dalloc(&p->fd_tw, (size_t)p->fd_np * sizeof(float2), tot) != hipSuccess ||
        dalloc(&p->fd_spec, (size_t)M * p->fd_np * sizeof(float2), tot) != hipSuccess ||
        dalloc(&p->fd_E, (size_t)bu * M * p->rows_p * sizeof(float2), tot) != hipSuccess)) ||
      (p->kt &&
       (dalloc(&p->kt_spec, (size_t)M * p->fd_np * sizeof(float2), tot) != hipSuccess ||
        dalloc(&p->kt_invd, (size_t)p->fd_np * sizeof(double), tot) != hipSuccess)) ||
      dalloc(&p->u_off, (size_t)bu * p->Mp * sizeof(int32_t), tot) != hipSuccess ||
      dalloc(&p->u_psi, (size_t)bu * p->Mp * sizeof(float2), tot) != hipSuccess ||
      dalloc((char **)&p->Gbuf[0], 2 * (size_t)bu * per_unit, tot) != hipSuccess ||
      dalloc(&p->packed, (size_t)p->batch_cells * p->rows * 8, tot) != hipSuccess ||
      dalloc((char **)&p->det_ws, p->det_ws_bytes, tot) != hipSuccess ||
      dalloc(&p->adj_ws, p->adj_ws_bytes, tot) != hipSuccess ||
      dalloc(&p->g_shift, 256, tot) != hipSuccess) {
    (void)hipGetLastError();
    release(p);
    return DSGRFT_E_NOMEM;
  }
  p->ws_bytes = tot;
  p->Gbuf[1] = (char *)p->Gbuf[0] + (size_t)bu * per_unit;
  p->gscbuf[1] = p->gscbuf[0] + (size_t)bu * p->rows_p;
  p->G = p->Gbuf[0];
  p->g_scale = p->gscbuf[0];
  if (hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_start, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_g[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_g[1], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_f[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_f[1], hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    release(p);
    return DSGRFT_E_DEVICE;
  }
  if (p->fft_tw) p->fft_chirp = p->fft_tw + M;
  if (p->FBs > 0) {
    std::vector<int32_t> cols(2 * sym_cols_n, -1);
    for (size_t c = 0; c < sym_plus.size(); ++c) {
      cols[c] = sym_plus[c];
      cols[sym_cols_n + c] = sym_minus[c];
    }
    if (hipMemcpy(p->sym_cols, cols.data(), cols.size() * sizeof(int32_t),
                  hipMemcpyHostToDevice) != hipSuccess) {
      release(p);
      return DSGRFT_E_DEVICE;
    }
  }
  if ((!p->kt && launch_fine_tables(p, nullptr) != hipSuccess) ||
      (p->FBs > 0 && launch_sym_table(p, nullptr) != hipSuccess) ||
      (p->fft_tw && launch_fft_tables(p, nullptr) != hipSuccess) ||
      (p->fd && launch_fd_twiddles(p, nullptr) != hipSuccess) ||
      (p->kt && launch_kt_tables(p, nullptr) != hipSuccess) ||
      hipDeviceSynchronize() != hipSuccess) {
    release(p);
    return DSGRFT_E_DEVICE;
  }
  *out = p;
  return DSGRFT_OK;
}

static void prof_free(dsgrft_plan p);

void dsgrft_plan_destroy(dsgrft_plan plan) {
  if (!plan) return;
  (void)hipDeviceSynchronize();
  prof_free(plan);
  release(plan);
}

dsgrft_status dsgrft_plan_get_info(dsgrft_plan p, dsgrft_plan_info *o) {
  if (!p || !o) return DSGRFT_E_INVALID;
  o->R = p->R;
  for (int q = 0; q < 3; ++q) {
    o->K[q] = p->K[q];
    o->i_lo[q] = p->ilo[q];
    o->step[q] = p->step[q];
  }
  o->K[0] = p->gK0;
  o->i_lo[0] = p->gilo0;
  o->kt_q_lo = p->kt ? p->kt_q_lo : 0;
  o->kt_folds = p->kt ? p->kt_na : 0;
  o->rows = p->rows;
  o->n_coarse = p->n_coarse;
  o->n_fine = p->n_fine;
  o->lambda = p->lam;
  o->dr = p->dr;
  o->T = p->T;
  o->workspace_bytes = p->ws_bytes;
  o->fd_pad = p->fd ? p->fd_np : 0;
  return DSGRFT_OK;
}

dsgrft_status dsgrft_coarse_tables(dsgrft_plan p, int64_t cc_begin, int64_t n,
                                   int32_t *d_off, void *d_psi, void *stream) {
  if (!p || !d_off || !d_psi || n < 1 || cc_begin < 0 || cc_begin + n > p->n_coarse)
    return DSGRFT_E_INVALID;
  if (p->kt) return DSGRFT_E_UNSUPPORTED;
  if (!on_plan_device(p)) return DSGRFT_E_INVALID;
  DS_TRY(launch_coarse_tables(p, cc_begin, n, p->M, d_off, (float2 *)d_psi,
                              (hipStream_t)stream));
  return DSGRFT_OK;
}

dsgrft_status dsgrft_mgift(dsgrft_plan p, const void *d_echo, int64_t cc_begin,
                           int64_t n, void *d_out, void *stream) {
  if (!p || !d_echo || !d_out || n < 1 || cc_begin < 0 || cc_begin + n > p->n_coarse)
    return DSGRFT_E_INVALID;
  if (!on_plan_device(p)) return DSGRFT_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  if (p->fd) DS_TRY(launch_range_fft(p, (const float2 *)d_echo, s));
  if (p->kt) DS_TRY(launch_keystone(p, s));
  const GatherSrc src = gather_src(p, (const float2 *)d_echo);
  for (int64_t c0 = 0; c0 < n; c0 += p->batch_units) {
    const int64_t nc = (n - c0) < p->batch_units ? (n - c0) : p->batch_units;
    DS_TRY(launch_coarse_tables(p, cc_begin + c0, nc, p->Mp, p->u_off, p->u_psi, s,
                                p->fd != 0));
    if (p->kt)
      DS_TRY(launch_kt_shift(p, nullptr, cc_begin + c0, 0, nc, s));
    else if (p->fd)
      DS_TRY(launch_fd_shift(p, nullptr, cc_begin + c0, 0, nc, 1, s));
    DS_TRY(launch_mgift_out(p, src, nc,
                            (float2 *)d_out + c0 * (int64_t)p->M * p->rows, s));
  }
  return DSGRFT_OK;
}

dsgrft_status dsgrft_search(dsgrft_plan p, dsgrft_form form, int32_t split,
                            const void *d_echo, const int64_t *d_cells,
                            int64_t cc_begin, int64_t n, float *d_pmax,
                            int32_t *d_argf, void *stream) {
  if (!p || !d_echo || !d_pmax || !d_argf || n < 1) return DSGRFT_E_INVALID;
  if (!d_cells && (cc_begin < 0 || cc_begin + n > p->n_coarse)) return DSGRFT_E_INVALID;
  dsgrft_status st = check_form(p, form, split);
  if (st != DSGRFT_OK) return st;
  if (!on_plan_device(p)) return DSGRFT_E_INVALID;
  return run_search(p, form, split, (const float2 *)d_echo, d_cells, cc_begin, n,
                    d_pmax, d_argf, nullptr, (hipStream_t)stream);
}

dsgrft_status dsgrft_search_full(dsgrft_plan p, dsgrft_form form, int32_t split,
                                 const void *d_echo, int64_t cc_begin, int64_t n,
                                 float *d_power, void *stream) {
  if (!p || !d_echo || !d_power || n < 1 || cc_begin < 0 || cc_begin + n > p->n_coarse)
    return DSGRFT_E_INVALID;
  if ((double)n * p->rows * (double)p->n_fine > 2147483647.0) return DSGRFT_E_INVALID;
  dsgrft_status st = check_form(p, form, split);
  if (st != DSGRFT_OK) return st;
  if (!on_plan_device(p)) return DSGRFT_E_INVALID;
  return run_search(p, form, split, (const float2 *)d_echo, nullptr, cc_begin, n,
                    nullptr, nullptr, d_power, (hipStream_t)stream);
}

dsgrft_status dsgrft_grft(dsgrft_plan p, const void *d_echo, int64_t cc_begin,
                          int64_t n, float *d_pmax, int32_t *d_argf, float *d_power,
                          void *stream) {
  if (!p || !d_echo || n < 1 || cc_begin < 0 || cc_begin + n > p->n_coarse)
    return DSGRFT_E_INVALID;
  if ((d_pmax == nullptr) != (d_argf == nullptr)) return DSGRFT_E_INVALID;
  if (!d_pmax && !d_power) return DSGRFT_E_INVALID;
  if (d_power && (double)n * p->rows * (double)p->n_fine > 2147483647.0)
    return DSGRFT_E_INVALID;
  if (p->kt) return DSGRFT_E_UNSUPPORTED;
  if (!on_plan_device(p)) return DSGRFT_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  const float2 *echo = (const float2 *)d_echo;
  for (int64_t c0 = 0; c0 < n; c0 += p->batch_cells) {
    const int64_t nc = (n - c0) < p->batch_cells ? (n - c0) : p->batch_cells;
    DS_TRY(launch_fill_u64(p->packed, nc * p->rows, s));
    DS_TRY(launch_grft(p, echo, cc_begin + c0, nc,
                       d_power ? d_power + c0 * p->rows * p->n_fine : nullptr, s));
    if (d_pmax)
      DS_TRY(launch_unpack(p, nc, d_pmax + c0 * p->rows, d_argf + c0 * p->rows, s));
  }
  return DSGRFT_OK;
}

dsgrft_status dsgrft_noise_power(dsgrft_plan p, const void *d_echo, double *d_sigma2,
                                 void *stream) {
  if (!p || !d_echo || !d_sigma2) return DSGRFT_E_INVALID;
  if (!on_plan_device(p)) return DSGRFT_E_INVALID;
  DS_TRY(launch_noise_power(p, (const float2 *)d_echo, d_sigma2, (hipStream_t)stream));
  return DSGRFT_OK;
}

// Count readback of the detection calls: with h_count set, wait for the
// stream, store the count and report E_CAPACITY when it exceeds cap.
static dsgrft_status read_count(const int32_t *d_count, int32_t cap, int32_t *h_count,
                                hipStream_t s) {
  if (!h_count) return DSGRFT_OK;
  int32_t c = 0;
  DS_TRY(hipMemcpyAsync(&c, d_count, sizeof(c), hipMemcpyDeviceToHost, s));
  DS_TRY(hipStreamSynchronize(s));
  *h_count = c;
  return c > cap ? DSGRFT_E_CAPACITY : DSGRFT_OK;
}

dsgrft_status dsgrft_lrt_threshold(dsgrft_plan p, double sigma2, double pfa,
                                   double *h_gamma2) {
  if (!p || !h_gamma2 || !std::isfinite(sigma2) || sigma2 < 0.0 || !(pfa > 0.0) ||
      !(pfa < 1.0))
    return DSGRFT_E_INVALID;
  *h_gamma2 = (-(double)p->M * sigma2) * std::log(pfa);
  return DSGRFT_OK;
}

dsgrft_status dsgrft_detect(dsgrft_plan p, const float *d_pmax, const int32_t *d_argf,
                            const int64_t *d_cells, int64_t cc_begin, int64_t n,
                            double sigma2, const double *d_sigma2, double pfa,
                            dsgrft_peak *d_peaks, int32_t cap, int32_t *d_count,
                            dsgrft_peak *d_best, int32_t *h_count, void *stream) {
  if (!p || !d_pmax || !d_argf || !d_count || n < 1 || cap < 0) return DSGRFT_E_INVALID;
  if (cap > 0 && !d_peaks) return DSGRFT_E_INVALID;
  if (!d_sigma2 && (!std::isfinite(sigma2) || sigma2 < 0.0)) return DSGRFT_E_INVALID;
  if (!(pfa > 0.0) || !(pfa < 1.0)) return DSGRFT_E_INVALID;
  if (!d_cells && (cc_begin < 0 || cc_begin + n > p->n_coarse)) return DSGRFT_E_INVALID;
  if (n > p->n_coarse || (double)n * p->rows > 2147483647.0) return DSGRFT_E_INVALID;
  if (!on_plan_device(p)) return DSGRFT_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  DS_TRY(launch_detect(p, d_pmax, d_argf, d_cells, cc_begin, n, sigma2, d_sigma2,
                       std::log(pfa), d_peaks, cap, d_count, d_best, s));
  return read_count(d_count, cap, h_count, s);
}

dsgrft_status dsgrft_detect_cfar(dsgrft_plan p, const float *d_pmax,
                                 const int32_t *d_argf, const int64_t *d_cells,
                                 int64_t cc_begin, int64_t n, int32_t guard, int32_t train,
                                 double alpha, dsgrft_peak *d_peaks, int32_t cap,
                                 int32_t *d_count, dsgrft_peak *d_best, int32_t *h_count,
                                 void *stream) {
  if (!p || !d_pmax || !d_argf || !d_count || n < 1 || cap < 0) return DSGRFT_E_INVALID;
  if (cap > 0 && !d_peaks) return DSGRFT_E_INVALID;
  if (guard < 0 || train < 1 || guard > 65536 || train > 65536) return DSGRFT_E_INVALID;
  if (!std::isfinite(alpha) || alpha < 0.0) return DSGRFT_E_INVALID;
  if (!d_cells && (cc_begin < 0 || cc_begin + n > p->n_coarse)) return DSGRFT_E_INVALID;
  if (n > p->n_coarse || (double)n * p->rows > 2147483647.0) return DSGRFT_E_INVALID;
  if (!on_plan_device(p)) return DSGRFT_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  DS_TRY(launch_detect_cfar(p, d_pmax, d_argf, d_cells, cc_begin, n, guard, train, alpha,
                            d_peaks, cap, d_count, d_best, s));
  return read_count(d_count, cap, h_count, s);
}

dsgrft_status dsgrft_adjoint_forward(dsgrft_plan p, const void *d_echo,
                                     const double *d_theta, int32_t B, double *d_J,
                                     double *d_saved, void *stream) {
  if (!p || !d_echo || !d_theta || !d_J || B < 1) return DSGRFT_E_INVALID;
  if (p->P > 2 || p->kt) return DSGRFT_E_UNSUPPORTED;
  if (!on_plan_device(p)) return DSGRFT_E_INVALID;
  DS_TRY(launch_adjoint_forward(p, (const float2 *)d_echo, d_theta, B, d_J, d_saved,
                                (hipStream_t)stream));
  return DSGRFT_OK;
}

dsgrft_status dsgrft_adjoint_backward(dsgrft_plan p, const void *d_echo,
                                      const double *d_theta, int32_t B,
                                      const double *d_saved, const double *d_gJ,
                                      double *d_grad_theta, void *d_grad_echo,
                                      void *stream) {
  if (!p || !d_echo || !d_theta || !d_saved || !d_gJ || B < 1) return DSGRFT_E_INVALID;
  if (!d_grad_theta && !d_grad_echo) return DSGRFT_E_INVALID;
  if (p->P > 2 || p->kt) return DSGRFT_E_UNSUPPORTED;
  if (!on_plan_device(p)) return DSGRFT_E_INVALID;
  DS_TRY(launch_adjoint_backward(p, (const float2 *)d_echo, d_theta, B, d_saved, d_gJ,
                                 d_grad_theta, (float2 *)d_grad_echo,
                                 (hipStream_t)stream));
  return DSGRFT_OK;
}

dsgrft_status dsgrft_refine(dsgrft_plan p, const void *d_echo, double *d_theta,
                            int32_t B, int32_t iters, double *d_J, void *stream) {
  if (!p || !d_echo || !d_theta || !d_J || B < 1 || iters < 0 || iters > 10000)
    return DSGRFT_E_INVALID;
  if (p->P > 2 || p->kt) return DSGRFT_E_UNSUPPORTED;
  if (!on_plan_device(p)) return DSGRFT_E_INVALID;
  DS_TRY(launch_refine(p, (const float2 *)d_echo, d_theta, B, iters, d_J,
                       (hipStream_t)stream));
  return DSGRFT_OK;
}

static void prof_free(dsgrft_plan p) {
  auto &pr = p->prof;
  for (int i = 0; i < 2 * pr.cap; ++i) {
    if (pr.ev_g && pr.ev_g[i]) (void)hipEventDestroy(pr.ev_g[i]);
    if (pr.ev_f && pr.ev_f[i]) (void)hipEventDestroy(pr.ev_f[i]);
  }
  std::free(pr.ev_g);
  std::free(pr.ev_f);
  pr = dsgrft_plan_s::Prof();
}

dsgrft_status dsgrft_profile_begin(dsgrft_plan p, int32_t capacity) {
  if (!p || capacity < 1 || capacity > (1 << 20)) return DSGRFT_E_INVALID;
  if (!on_plan_device(p)) return DSGRFT_E_INVALID;
  prof_free(p);
  auto &pr = p->prof;
  pr.ev_g = (hipEvent_t *)std::calloc(2 * (size_t)capacity, sizeof(hipEvent_t));
  pr.ev_f = (hipEvent_t *)std::calloc(2 * (size_t)capacity, sizeof(hipEvent_t));
  if (!pr.ev_g || !pr.ev_f) {
    prof_free(p);
    return DSGRFT_E_NOMEM;
  }
  pr.cap = capacity;
  for (int i = 0; i < 2 * capacity; ++i) {
    if (hipEventCreate(&pr.ev_g[i]) != hipSuccess ||
        hipEventCreate(&pr.ev_f[i]) != hipSuccess) {
      prof_free(p);
      return DSGRFT_E_DEVICE;
    }
  }
  return DSGRFT_OK;
}

dsgrft_status dsgrft_profile_end(dsgrft_plan p, dsgrft_profile *out) {
  if (!p || !out) return DSGRFT_E_INVALID;
  auto &pr = p->prof;
  std::memset(out, 0, sizeof(*out));
  if (pr.cap == 0) return DSGRFT_E_INVALID;
  if (hipDeviceSynchronize() != hipSuccess) {
    prof_free(p);
    return DSGRFT_E_DEVICE;
  }
  double gms = 0.0, fms = 0.0;
  for (int i = 0; i < pr.ng; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pr.ev_g[2 * i], pr.ev_g[2 * i + 1]) != hipSuccess) {
      prof_free(p);
      return DSGRFT_E_DEVICE;
    }
    gms += ms;
  }
  for (int i = 0; i < pr.nf; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pr.ev_f[2 * i], pr.ev_f[2 * i + 1]) != hipSuccess) {
      prof_free(p);
      return DSGRFT_E_DEVICE;
    }
    fms += ms;
  }
  out->gather_launches = pr.ng;
  out->fine_launches = pr.nf;
  out->gather_ms = gms;
  out->fine_ms = fms;
  out->gather_bytes = pr.gbytes;
  out->fine_flops = pr.fflops;
  out->fine_cell_pulses = pr.fcp;
  out->fine_mfma_flops = pr.fxflops;
  prof_free(p);
  return DSGRFT_OK;
}

}  // extern "C"
