// Internal declarations of the DS-GRFT library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsgrft.h"

// ---------------------------------------------------------------------------
// Exact lattice arithmetic, shared by host plan code and device kernels.
//
// With integer fine-lattice indices i = (i1, i2, i3) and t_m = m / PRF:
//   2 D(t_m) / lambda = Num / M^3,  D(t_m) / dr = Num / (R M^3),
//   Num(m; i) = i1 m M^2 + i2 m^2 M + i3 m^3.
// The range offset is round-half-up of Num / (R M^3) and the phase is
// exp(+j 2 pi (Num mod M^3) / M^3), both from exact integers.
// ---------------------------------------------------------------------------
struct Lat {
  int64_t M, M3, RM3;  // M, M^3, R * M^3
};

__host__ __device__ inline int64_t lat_num(const Lat &L, int64_t m, int64_t i1,
                                           int64_t i2, int64_t i3) {
  return i1 * m * L.M * L.M + i2 * m * m * L.M + i3 * m * m * m;
}

__host__ __device__ inline int64_t floor_div(int64_t a, int64_t b) {  // b > 0
  int64_t q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}

__host__ __device__ inline int32_t lat_offset(const Lat &L, int64_t num) {
  return (int32_t)floor_div(2 * num + L.RM3, 2 * L.RM3);
}

// (Num mod M^3) / M^3 * 2 as the argument of sincospi.
__host__ __device__ inline double lat_turns2(const Lat &L, int64_t num) {
  int64_t r = num % L.M3;
  if (r < 0) r += L.M3;
  return 2.0 * (double)r / (double)L.M3;
}

__device__ inline float2 lat_phasor(const Lat &L, int64_t num) {
  double s, c;
  sincospi(lat_turns2(L, num), &s, &c);
  return make_float2((float)c, (float)s);
}

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
enum { KTILE = 64 };      // pulses are padded to a multiple of this
enum { ROWTILE = 256 };   // range rows are padded to a multiple of this
enum { COLTILE = 128 };   // fine-search columns padded to a multiple of this

struct dsgrft_plan_s {
  dsgrft_radar radar;
  dsgrft_config cfg;
  int device;
  int M, N, P, n_begin, n_end, rows;
  int R, h;
  int K[3], ilo[3];     // coarse lattice the kernels walk (see S0)
  int S0;               // axis-0 coarse step: R, or M for DS-KT-MFP
  int gK0, gilo0;       // axis 0 of the DS-GRFT lattice (reported in the info)
  int64_t n_coarse, n_fine;
  int C;    // fine-search columns per gathered unit: R^min(P, 2)
  int R3;   // gathered units per coarse cell: R for P = 3, else 1
  double lam, dr, T, step[3];
  Lat lat;
  // padded sizes
  int Mp, rows_p, Cp, KB, NB, FB;
  int64_t batch_units, batch_cells;
  // device buffers owned by the plan
  float2 *F32;          // [Mp][Cp] fine phasors, complex64
  uint4 *F16;           // MFMA fragments, 4 planes (re_hi, im_hi, re_lo, im_lo)
  uint4 *FBF16;         // same in bf16
  uint4 *F8;            // e4m3 fragments (K blocks of 64), same 4 planes
  int FBs;              // column blocks of the conjugate-pair table (even)
  uint4 *FS16;          // its fp16 fragments, 2 planes (re, im) x FBs blocks
  uint4 *FSB16;         // the same columns in bf16, 4 planes (re/im hi, re/im lo)
  uint4 *FS8;           // the same columns in e4m3, 4 planes (null without F8)
  int32_t *sym_cols;    // [2][FBs * 32]: fine cell of +d and of -d per
                        //   column (-1: none)
  int32_t *u_off;       // [batch_units][Mp] unit range offsets
  float2 *u_psi;        // [batch_units][Mp] unit de-ramp phasors
  void *G;              // gathered batch being produced or consumed (a slot
                        //   of Gbuf), max 8 bytes per (unit,row,pulse)
  int32_t *g_scale;     // [batch_units][rows_p] per-row E8M0 codes of that slot
  int32_t *g_shift;     // [2]: largest |Re|/|Im| echo component (float bits)
                        //   and the fp16 forms' power-of-two shift of G
  void *Gbuf[2];        // two slots: batch b + 1 is gathered while the fine
  int32_t *gscbuf[2];   //   search reads batch b
  hipStream_t aux;      // producer stream of the search pipeline (tables,
                        //   coarse compensation, gathers); default priority
  hipEvent_t ev_start, ev_g[2], ev_f[2];  // ordering events of the pipeline
  float2 *fft_tw;       // [M] exp(+j 2 pi k / M) (FFT form; null if unsupported)
  float2 *fft_chirp;    // [R or 1][M] fine-acceleration chirps (FFT form)
  // frequency-domain mGIFT (cfg.mgift == 1)
  int fd;               // 1: frequency-domain coarse compensation
  int fd_np;            // padded range-FFT length
  float2 *fd_tw;        // [fd_np] exp(+j 2 pi k / fd_np)
  float2 *fd_spec;      // [M][fd_np] range spectrum of the current echo
  float2 *fd_E;         // [batch_units][M][rows_p] shifted rows
  // DS-KT-MFP (cfg.mgift == 2; fd is 1 as well)
  int kt;
  int kt_q_lo, kt_na;   // folding factors q_lo .. q_lo + kt_na - 1
  float2 *kt_spec;      // [M][fd_np] keystone-transformed spectrum
  double *kt_invd;      // [fd_np] 1 / (R fd_np + k_s)
  unsigned long long *packed;  // [batch_cells][rows] (power bits, ~fine)
  void *det_ws;         // detection partials
  size_t det_ws_bytes;
  double *adj_ws;       // adjoint scratch
  size_t adj_ws_bytes;
  size_t ws_bytes;
  // measurement hook (dsgrft_profile_begin / _end)
  struct Prof {
    int cap = 0;
    int ng = 0, nf = 0;
    hipEvent_t *ev_g = nullptr, *ev_f = nullptr;  // [2 * cap] each
    double gbytes = 0.0, fflops = 0.0, fcp = 0.0, fxflops = 0.0;
  } prof;
};

// Cell id of the i-th listed cell.
__device__ inline int64_t cell_id(const int64_t *cells, int64_t base, int64_t i) {
  return cells ? cells[i] : base + i;
}

// Coarse centre indices of cell k.  Axis 0 steps by S0 fine indices (R on
// the DS-GRFT lattice, M on the folded velocity lattice of DS-KT-MFP, whose
// centre q M is the folding factor), the other axes by R.
__host__ __device__ inline void coarse_centre(const int *K, const int *ilo, int R,
                                              int P, int64_t k, int64_t ic[3],
                                              int S0) {
  int64_t k1 = k % K[0];
  int64_t k2 = (k / K[0]) % K[1];
  int64_t k3 = k / ((int64_t)K[0] * K[1]);
  int64_t kk[3] = {k1, k2, k3};
  for (int p = 0; p < 3; ++p) {
    const int S = p == 0 ? S0 : R;
    ic[p] = (p < P) ? (int64_t)ilo[p] + kk[p] * S + S / 2 : 0;
  }
}

// Fine offsets of flat fine index f (axis 0 has S0 cells, the others R).
__host__ __device__ inline void fine_offsets(int R, int P, int64_t f, int64_t fo[3],
                                             int S0) {
  int64_t u = f;
  for (int p = 0; p < 3; ++p) {
    const int S = p == 0 ? S0 : R;
    fo[p] = (p < P) ? (u % S) - S / 2 : 0;
    u /= S;
  }
}

// ---------------------------------------------------------------------------
// Launch helpers (implemented in the .hip files)
// ---------------------------------------------------------------------------
#define DS_TRY(expr)                                     \
  do {                                                   \
    if ((expr) != hipSuccess) return DSGRFT_E_DEVICE;    \
  } while (0)

hipError_t launch_fine_tables(dsgrft_plan p, hipStream_t s);
hipError_t launch_sym_table(dsgrft_plan p, hipStream_t s);
hipError_t launch_unit_tables(dsgrft_plan p, const int64_t *cells,
                              int64_t cc_base, int64_t unit0, int64_t nunits,
                              hipStream_t s);
hipError_t launch_coarse_tables(dsgrft_plan p, int64_t cc_begin, int64_t n,
                                int stride, int32_t *off, float2 *psi,
                                hipStream_t s, bool zero_off = false);
size_t detect_ws_bytes(int64_t max_entries);
// Where the gathers read: the echo ([M][N], window from n_begin) or, in the
// frequency-domain mode, the shifted rows of each unit ([u][M][rows_p]).
// Forms whose gathered rows are fp16 (scaled by the echo shift).
inline bool fp16_form(dsgrft_form f) {
  return f == DSGRFT_FORM_F16 || f == DSGRFT_FORM_F16_3M || f == DSGRFT_FORM_F16_SYM;
}

struct GatherSrc {
  const float2 *echo;
  int N, n_begin;
  int64_t unit_stride;
};
GatherSrc gather_src(dsgrft_plan p, const float2 *echo);
hipError_t launch_gather_f32(dsgrft_plan p, GatherSrc src, int64_t nunits,
                             hipStream_t s);
hipError_t launch_echo_shift(dsgrft_plan p, const float2 *echo, hipStream_t s);
hipError_t launch_gather_lp(dsgrft_plan p, dsgrft_form form, int split,
                            GatherSrc src, int64_t nunits, hipStream_t s);
hipError_t launch_mgift_out(dsgrft_plan p, GatherSrc src, int64_t nunits,
                            float2 *out, hipStream_t s);
int fd_pad_length(dsgrft_plan p);
hipError_t launch_fd_twiddles(dsgrft_plan p, hipStream_t s);
hipError_t launch_range_fft(dsgrft_plan p, const float2 *echo, hipStream_t s);
hipError_t launch_fd_shift(dsgrft_plan p, const int64_t *cells, int64_t cc_base,
                           int64_t unit0, int64_t nunits, int R3, hipStream_t s);
hipError_t launch_kt_tables(dsgrft_plan p, hipStream_t s);
hipError_t launch_keystone(dsgrft_plan p, hipStream_t s);
hipError_t launch_kt_shift(dsgrft_plan p, const int64_t *cells, int64_t cc_base,
                           int64_t unit0, int64_t nunits, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *ptr, int64_t n, hipStream_t s);
hipError_t launch_fine_f32(dsgrft_plan p, int64_t nunits, int64_t unit0,
                           float *full, int64_t full_cell0, hipStream_t s);
hipError_t launch_fine_mfma(dsgrft_plan p, dsgrft_form form, int split,
                            int64_t nunits, int64_t unit0, float *full,
                            hipStream_t s);
bool fft_form_supported(int M);
size_t fft_table_elems(int M, int R, int P);
hipError_t launch_fft_tables(dsgrft_plan p, hipStream_t s);
hipError_t launch_fine_fft(dsgrft_plan p, int64_t nunits, int64_t unit0,
                           float *full, hipStream_t s);
hipError_t launch_unpack(dsgrft_plan p, int64_t ncells, float *pmax,
                         int32_t *argf, hipStream_t s);
hipError_t launch_grft(dsgrft_plan p, const float2 *echo, int64_t cc_begin,
                       int64_t n, float *full, hipStream_t s);
hipError_t launch_noise_power(dsgrft_plan p, const float2 *echo, double *out,
                              hipStream_t s);
hipError_t launch_detect(dsgrft_plan p, const float *pmax, const int32_t *argf,
                         const int64_t *cells, int64_t cc_begin, int64_t n,
                         double sigma2, const double *d_sigma2, double ln_pfa,
                         dsgrft_peak *peaks, int32_t cap, int32_t *count,
                         dsgrft_peak *best, hipStream_t s);
hipError_t launch_detect_cfar(dsgrft_plan p, const float *pmax, const int32_t *argf,
                              const int64_t *cells, int64_t cc_begin, int64_t n, int guard,
                              int train, double alpha, dsgrft_peak *peaks, int32_t cap,
                              int32_t *count, dsgrft_peak *best, hipStream_t s);
hipError_t launch_adjoint_forward(dsgrft_plan p, const float2 *echo,
                                  const double *theta, int B, double *J,
                                  double *saved, hipStream_t s);
hipError_t launch_adjoint_backward(dsgrft_plan p, const float2 *echo,
                                   const double *theta, int B,
                                   const double *saved, const double *gJ,
                                   double *grad_theta, float2 *grad_echo,
                                   hipStream_t s);
hipError_t launch_refine(dsgrft_plan p, const float2 *echo, double *theta, int B,
                         int iters, double *J, hipStream_t s);
