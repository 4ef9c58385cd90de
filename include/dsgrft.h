/*
 * dsgrft.h -- C ABI of the MI355X dual-scale GRFT search library.
 *
 * Method: Li et al., "Efficient dual-scale generalized Radon-Fourier transform
 * detector family for long time coherent integration" (arXiv 2403.06788).
 *
 * Problem (Sec. V-A, Alg. 3): a range-compressed complex echo s[m][n]
 * (M pulses x N range bins), radar parameters (f_c, f_s, PRF) and motion
 * parameter extents go in; a detection map and peak parameters come out.
 * The search evaluates, for every coarse cell c_c of the dual-scale lattice
 * (Sec. IV-B, eqs. (48)-(52)), the mGIFT (eqs. (46)-(47), Alg. 1: by default
 * in the time domain, a gather of each pulse's range bin along the coarse
 * walk and the pre-DFM de-ramp; optionally in the frequency domain) followed
 * by the GFT over the cell's fine space (eq. (44), Alg. 2, as a GEMM or as a
 * slow-time FFT), and reduces |.|^2 over the fine space (eq. (72)).
 *
 * Conventions shared by every entry point
 *  - Complex data are interleaved (re, im) pairs: complex64 = 2 x float,
 *    complex128 = 2 x double.  The echo is row-major [M][N] complex64.
 *  - "d_" arguments are device pointers on the current HIP device; "h_"
 *    arguments are host pointers.  The caller owns every I/O buffer.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *    device work is ordered on it; no entry point synchronises the stream
 *    unless its comment says so.  dsgrft_search and dsgrft_search_full also
 *    run part of their work on a second stream owned by the plan; that work
 *    starts after everything enqueued on `stream` before the call and
 *    finishes before anything enqueued on `stream` after it.  A plan may be
 *    used by one stream at a time.
 *  - The plan owns its device workspace, allocated in dsgrft_plan_create.
 *    Execution entry points allocate nothing.
 *  - Errors are reported as status codes only; nothing aborts or prints.
 *    On any non-OK status no device work has been enqueued, except for
 *    DSGRFT_E_DEVICE, where a HIP call failed part-way.
 *
 * Lattice (reading of eqs. (39)-(42) with alpha_p = 1 per order):
 *  lambda = c/f_c, dr = c/(2 f_s), T = M/PRF, R = f_c/f_s (must be an
 *  integer), fine steps dv = lambda/(2T), da = lambda/T^2, dj = 3 lambda/T^3
 *  (motion r(t) = r0 + v t + a t^2/2 + j t^3/6, t_m = m/PRF, m = 0..M-1).
 *  Axis p covers integer indices [i_lo,p, i_lo,p + K_p R) (bounds rounded
 *  outward; within 1e-6 of a lattice point counts as on it).  Coarse cell
 *  k = (k3 K2 + k2) K1 + k1 has centre i_c,p = i_lo,p + k_p R + R/2 (integer
 *  division); fine index f = (u3 R + u2) R + u1, offsets u_p - R/2.
 *  Range offsets round half up; all offsets and phases are exact integers.
 */
#ifndef DSGRFT_H
#define DSGRFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DSGRFT_OK = 0,
  DSGRFT_E_INVALID = 1,      /* invalid argument (null pointer, bad size, ...) */
  DSGRFT_E_NOMEM = 2,        /* device allocation failed (plan creation only)  */
  DSGRFT_E_DEVICE = 3,       /* a HIP runtime call failed                      */
  DSGRFT_E_UNSUPPORTED = 4,  /* valid request outside what is implemented      */
  DSGRFT_E_CAPACITY = 5      /* output list too small; true count reported     */
} dsgrft_status;

/* Arithmetic of the fine search (the GFT stage, eq. (44)).  FP32 runs on the
 * vector ALUs; the others on MFMA with FP32 accumulation.  Both operands (the
 * fine phasors F and the gathered rows G) are split as x = hi + lo, and
 * `split` (1..4) selects the products summed: 1: Fh Gh; 2: + Fl Gh;
 * 3: + Fh Gl; 4: + Fl Gl.
 * FP8 is OCP e4m3 with power-of-two block scales: F is stored as
 * e4m3(256 F) (lo: e4m3(16 (256 F - hi))), and every (gathered unit, range
 * row) gets the scale 2^(8-e) where 2^(e-1) <= the row's largest |Re|/|Im|
 * echo component < 2^e.  Echo components must stay below 2^100 in
 * magnitude for this form.
 * The fp16 forms (F16, F16_3M, F16_SYM) store the gathered rows times 2^sh,
 * one shift per echo that puts its largest |Re|/|Im| component in
 * [2^9, 2^10) (clamped to |sh| <= 100), and scale the power back by
 * 2^(-2 sh); bf16 and FP32 keep FP32's exponent range.  So every form takes
 * any finite echo whose powers stay inside the FP32 range, and its map
 * scales exactly with the echo by powers of two. */
typedef enum {
  DSGRFT_FORM_F32 = 0,   /* plain FP32 (speed baseline), split 1    */
  DSGRFT_FORM_F16 = 1,   /* fp16 x fp16 -> fp32, split 1..4         */
  DSGRFT_FORM_BF16 = 2,  /* bf16 x bf16 -> fp32, split 1..4         */
  DSGRFT_FORM_FP8 = 3,   /* e4m3 x e4m3 (scaled) -> fp32, split 1..4 */
  DSGRFT_FORM_F32_FFT = 4, /* FP32, fine velocities by a slow-time FFT as in
                              Alg. 2 (one per fine acceleration); split 1;
                              M a power of two in [64, 2048], else
                              E_UNSUPPORTED; the only form of DS-KT-MFP */
  DSGRFT_FORM_F16_3M = 5,  /* fp16, split 1, each complex product from three
                              real MFMA products (Gauss): P1 = Fr Gr,
                              P2 = Fi Gi, P3 = (Fr + Fi)(Gr + Gi) with the
                              sums rounded to fp16; Re = P1 - P2,
                              Im = P3 - P1 - P2 (FP32) */
  DSGRFT_FORM_BF16_GLO = 6, /* bf16, split 2 only: Fh Gh + Fh Gl, the
                              gathered rows split into hi + lo and the fine
                              table not (the other order of split 2) */
  DSGRFT_FORM_F16_SYM = 7, /* fp16, split 1, the fine cells taken in
                              conjugate pairs: the fine offsets are symmetric
                              about the coarse centre and the fine phase
                              (eq. (44)) is linear in them, so the cell at
                              -d has the conjugate phasor of the cell at +d;
                              the four real products Fr Gr, Fi Gi, Fr Gi,
                              Fi Gr of the +d column give both cells.  Same
                              operands and rounding as F16 split 1; not for
                              DS-KT-MFP plans */
  DSGRFT_FORM_BF16_SYM = 8, /* bf16 over the conjugate pairs of F16_SYM,
                              split 2: Fh Gh + Fh Gl (the products of
                              BF16_GLO), split 3: + Fl Gh (those of BF16
                              split 3); every part accumulates into the same
                              four real products of a pair; not for
                              DS-KT-MFP plans */
  DSGRFT_FORM_FP8_SYM = 9  /* e4m3 over the conjugate pairs of F16_SYM with
                              the operands and block scales of FP8, split 3
                              (Fh Gh + Fl Gh + Fh Gl) or 4 (+ Fl Gl), every
                              part into the same four real products of a
                              pair; not for DS-KT-MFP plans */
} dsgrft_form;

typedef struct {
  double fc;     /* carrier frequency f_c [Hz]                          */
  double fs;     /* range sampling rate f_s [Hz]; range bin c/(2 f_s)   */
  double prf;    /* pulse repetition frequency [Hz]                     */
  double c;      /* propagation speed [m/s] (3e8 in the paper)          */
  double kappa;  /* scale of Prop. 1; only 1.0 is supported             */
} dsgrft_radar;

typedef struct {
  double min, max;  /* search extent: v [m/s], a [m/s^2], j [m/s^3] */
} dsgrft_axis;

typedef struct {
  int32_t M;          /* pulses                                           */
  int32_t N;          /* range bins of the echo                           */
  int32_t order;      /* motion order P in 1..3                           */
  int32_t n_begin;    /* first searched range row (paper's bins of        */
  int32_t n_end;      /*   interest, Sec. IV-E); 0,0 means [0, N)         */
  dsgrft_axis axis[3];/* extents of v, a, j (orders above P are ignored)  */
  int32_t batch;      /* gathered units per fine-search batch; 0 = auto   */
  int32_t mgift;      /* coarse compensation (mGIFT, Alg. 1):             */
                      /*   0: time domain, nearest range bin of the walk  */
                      /*   1: frequency domain, exp(+j 2 pi k_s x / N') on */
                      /*      the range spectrum zero-padded to N' (the   */
                      /*      smallest power of two >= N + walk bound),   */
                      /*      then IFFT; N' <= 16384 else E_UNSUPPORTED   */
                      /*   2: DS-KT-MFP (Alg. 4, Prop. 3): keystone       */
                      /*      transform of the same spectrum, then per    */
                      /*      coarse cell the folding-factor and coarse   */
                      /*      acceleration compensation of eq. (26) and   */
                      /*      IFFT; see "DS-KT-MFP plans" below           */
} dsgrft_config;

/* DS-KT-MFP plans (mgift = 2) need order 2 and M a power of two in
 * [64, 2048] (else E_UNSUPPORTED).  Their lattice folds the velocity axis
 * (eq. (23)): a fine velocity index is i1 = q M + i1', i1' in [-M/2, M/2),
 * with folding factors q = q_lo .. q_lo + n_fold - 1 covering the DS-GRFT
 * axis indices [i_lo,1, i_lo,1 + K1 R); the acceleration axis keeps the
 * DS-GRFT coarse cells.  Coarse cell k = k2 n_fold + (q - q_lo) (k2 < K2,
 * centre i2c = i_lo,2 + k2 R + R/2); fine index f = u2 M + u1, i1' = u1 -
 * M/2, acceleration index i2c + u2 - R/2, so n_fine = M R.  With the range
 * spectrum S[m][k] (length N' as in mode 1, signed index k_s) and
 * eps_k = k_s / (R N' + k_s):
 *   S_KT[m][k] = sum_{m'<M} S[m'][k] sinc(m - m' - m eps_k),
 *   y[m][r] = psi(m) (1/N') sum_k S_KT[m][k]
 *             exp(+j 2 pi (q m eps_k - k_s x2(m)/N' + k (n_begin + r)/N')),
 *   x2(m) = i2c m^2 / (R M^2), psi(m) = exp(+j 2 pi i2c m^2 M / M^3),
 *   Y[f][r] = sum_m y[m][r] exp(+j 2 pi (i1' m M^2 + (u2 - R/2) m^2 M) / M^3).
 * They support dsgrft_mgift (y), dsgrft_search / dsgrft_search_full with
 * DSGRFT_FORM_F32_FFT, dsgrft_detect and dsgrft_noise_power; the other forms
 * and entry points return E_UNSUPPORTED. */

typedef struct {
  int32_t R;             /* fine cells per coarse step and order          */
  int32_t K[3];          /* DS-GRFT coarse cells per order (1 above P)    */
  int32_t i_lo[3];       /* first fine lattice index per order            */
  int32_t rows;          /* n_end - n_begin                               */
  int64_t n_coarse;      /* K1 K2 K3 (DS-KT-MFP: n_fold K2)               */
  int64_t n_fine;        /* R^P (DS-KT-MFP: M R)                          */
  double lambda, dr, T;  /* wavelength, range bin, integration time       */
  double step[3];        /* fine steps dv, da, dj                         */
  size_t workspace_bytes;/* device memory held by the plan                */
  int32_t fd_pad;        /* N' of the frequency-domain mGIFT (0 if the    */
                         /*   plan uses the time-domain gather)           */
  int32_t kt_q_lo;       /* DS-KT-MFP: first folding factor (else 0)      */
  int32_t kt_folds;      /* DS-KT-MFP: folding factors n_fold (else 0);   */
                         /*   n_coarse = n_fold K2                         */
} dsgrft_plan_info;

typedef struct {
  int64_t coarse;  /* coarse cell index k                                 */
  int32_t row;     /* range row n0 (absolute bin index)                   */
  int32_t fine;    /* fine index f                                        */
  float power;     /* |Y|^2 at the cell                                   */
  float pad_;
  double r0, v, a, j; /* eq. (72) with kappa = 1: n0 dr, lattice * steps  */
} dsgrft_peak;

typedef struct dsgrft_plan_s *dsgrft_plan;

/* Plan creation: validates the radar and lattice, derives the dual-scale
 * lattice and builds the fine phase matrix H_DFM(t_m; c_f) x velocity term
 * (eq. (44)) for the orders 1..min(P,2) in every arithmetic form, and sizes
 * the workspace.  E_INVALID for null pointers, M or N < 1, order outside
 * 1..3, min > max, f_c/f_s not a positive integer, a trajectory numerator that
 * could leave int64, or a bad row range; E_UNSUPPORTED for kappa != 1;
 * E_NOMEM if device memory runs out.  Uses the current HIP device and
 * synchronises it before returning. */
dsgrft_status dsgrft_plan_create(const dsgrft_radar *radar,
                                 const dsgrft_config *cfg, dsgrft_plan *out);

/* Releases the plan and its workspace (synchronises the device first).
 * Accepts NULL. */
void dsgrft_plan_destroy(dsgrft_plan plan);

/* The plan's derived quantities (Sec. II-B and Sec. IV-B: wavelength, range
 * bin, integration time, the fine steps of eqs. (39)-(42) with alpha_p = 1,
 * the coarse cells per order of the dual-scale lattice, eqs. (48)-(52), and
 * the fine cells per coarse cell, eq. (52)), as defined in the header
 * comment and dsgrft_plan_info above.  Host-only; E_INVALID for NULL
 * arguments. */
dsgrft_status dsgrft_plan_get_info(dsgrft_plan plan, dsgrft_plan_info *out);

/* Static text for a status code (never NULL). */
const char *dsgrft_status_string(dsgrft_status s);

/* Coarse tables (stage a0 of the hot path): for coarse cells
 * [cc_begin, cc_begin + n): d_off[i][m] = round-half-up walk in bins of the
 * cell centre (mGIFT envelope correction, eq. (46)), d_psi[i][m] =
 * exp(+j 2 pi Num/M^3), the pre-DFM phase H_pre-DFM of eq. (47), complex64.
 * Layout [n][M].  The offsets are the nearest-bin walk whatever the plan's
 * mgift mode.  E_INVALID if the range leaves [0, n_coarse); E_UNSUPPORTED
 * for DS-KT-MFP plans. */
dsgrft_status dsgrft_coarse_tables(dsgrft_plan plan, int64_t cc_begin,
                                   int64_t n, int32_t *d_off, void *d_psi,
                                   void *stream);

/* mGIFT (stages a1 + a2, Alg. 1): for coarse cells [cc_begin, cc_begin + n)
 * writes y[i][m][r] as complex64, layout [n][M][rows].  Time-domain plans
 * (mgift = 0): y = S(m, n_begin + r + off) * psi (S = 0 outside [0, N)).
 * Frequency-domain plans (mgift = 1): y = psi * (1/N') sum_k S'[m][k]
 * exp(+j 2 pi k_s x(m) / N') exp(+j 2 pi k (n_begin + r) / N'), with S' the
 * range DFT of row m zero-padded to N', k_s the signed frequency index and
 * x(m) = Num(m) / (R M^3) the cell's walk in bins (H_RM of eq. (10)).
 * DS-KT-MFP plans (mgift = 2): the y of "DS-KT-MFP plans" above. */
dsgrft_status dsgrft_mgift(dsgrft_plan plan, const void *d_echo,
                           int64_t cc_begin, int64_t n, void *d_out,
                           void *stream);

/* DS-GRFT search (stages a1..a4, Alg. 3): for each listed coarse cell and
 * range row, the largest |Y|^2 over the cell's fine space and the smallest
 * fine index attaining it (ties to the smaller index).  Cells are
 * d_cells[0..n) (device int64 list, each in [0, n_coarse): other values
 * give unspecified results but no access outside the plan's and the
 * caller's buffers) or, when d_cells is NULL,
 * cc_begin..cc_begin+n-1.  Outputs d_pmax, d_argf: [n][rows] (float, int32).
 * `form`/`split`: see dsgrft_form; FP32, FFT, F16_3M and F16_SYM require split = 1,
 * BF16_GLO split = 2, BF16_SYM split 2 or 3 (else E_INVALID).  The echo must
 * stay unchanged until the stream reaches the end of this call. */
dsgrft_status dsgrft_search(dsgrft_plan plan, dsgrft_form form, int32_t split,
                            const void *d_echo, const int64_t *d_cells,
                            int64_t cc_begin, int64_t n, float *d_pmax,
                            int32_t *d_argf, void *stream);

/* Full DS-GRFT power map |Y|^2 for coarse cells [cc_begin, cc_begin + n):
 * d_power[n][rows][n_fine] float.  Same forms as dsgrft_search.  Intended for
 * small plans (tests, figures); E_INVALID if the map would exceed 2^31
 * elements. */
dsgrft_status dsgrft_search_full(dsgrft_plan plan, dsgrft_form form,
                                 int32_t split, const void *d_echo,
                                 int64_t cc_begin, int64_t n, float *d_power,
                                 void *stream);

/* Single-scale TD-GRFT (Sec. III-A-1, eq. (13)) at the same lattice points,
 * FP32: per-cell range offsets along the full walk.  d_pmax/d_argf as in
 * dsgrft_search for cells [cc_begin, cc_begin+n); d_power ([n][rows][n_fine]
 * float) may be NULL, otherwise it receives the full map. */
dsgrft_status dsgrft_grft(dsgrft_plan plan, const void *d_echo,
                          int64_t cc_begin, int64_t n, float *d_pmax,
                          int32_t *d_argf, float *d_power, void *stream);

/* Noise power sigma^2 of the LRT threshold (Sec. III-C, eq. (33)): the
 * threshold is written for the noise of the K range-frequency bins; on a
 * range-compressed echo those bins are folded into the per-sample noise
 * power, estimated here as the mean of |s[m][n]|^2 over all M N samples
 * (FP64 partial sums of 65536 samples, summed in a fixed order; the
 * estimator itself is not in the paper, and the targets' energy biases it
 * upward by their share of the total).  Writes one double to d_sigma2. */
dsgrft_status dsgrft_noise_power(dsgrft_plan plan, const void *d_echo,
                                 double *d_sigma2, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc), who
 * therefore cannot create a plan there either: dsgrft_noise_power without a
 * plan.  Same kernels, same summation order and so the same double as
 * dsgrft_noise_power on the same echo [M][N] (complex64, device); writes one
 * double to d_sigma2.  The partial sums (one per 65536 samples) live in a
 * static device array of DSGRFT_NOALLOC_MAX_PARTS doubles that each GPU the
 * library runs on holds until the process ends; M N above
 * 65536 * DSGRFT_NOALLOC_MAX_PARTS (2^28 samples) returns E_INVALID, as do
 * NULL pointers and M or N < 1.  Allocates nothing and does not
 * synchronise.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (different streams or threads) race; order them on one
 * stream. */
#define DSGRFT_NOALLOC_MAX_PARTS 4096
dsgrft_status dsgrft_noise_power_noalloc(const void *d_echo, int32_t M, int32_t N,
                                         double *d_sigma2, void *stream);

/* LRT threshold on |Y|^2 (Sec. III-C, eqs. (31), (33)): gamma^2 =
 * -M sigma^2 ln P_FA, evaluated in FP64 as (-M sigma^2) ln P_FA, the K
 * frequency bins of eq. (33) folded into sigma^2 (see dsgrft_noise_power).
 * Host-only.  E_INVALID unless sigma2 is finite and >= 0 and 0 < pfa < 1. */
dsgrft_status dsgrft_lrt_threshold(dsgrft_plan plan, double sigma2, double pfa,
                                   double *h_gamma2);

/* LRT detection (Sec. III-C, eqs. (31), (33); Alg. 3): entries of a reduced
 * map [n][rows] (cells cc_begin.. or d_cells as in dsgrft_search) with power
 * > gamma^2 = -M sigma^2 ln P_FA (FP64, as in dsgrft_lrt_threshold) are
 * listed in flat order (cell, then row) into d_peaks[0..cap) with their
 * parameters (eq. (72), kappa = 1).  sigma^2 is *d_sigma2 when d_sigma2 is
 * not NULL (a device double, e.g. written by dsgrft_noise_power earlier on
 * the same stream; a NaN there yields no detection), else `sigma2`.
 * *d_count (device) receives the number of entries above the threshold,
 * which may exceed cap (only the first cap are written).  d_best (device,
 * may be NULL) receives the global maximum (smallest flat index on ties),
 * whatever the threshold.
 * h_count: NULL, or a host int32.  When set, the call waits until `stream`
 * has completed, stores the count there and returns DSGRFT_E_CAPACITY if it
 * exceeds cap (the outputs are complete otherwise); when NULL the call does
 * not synchronise and cannot report overflow (compare *d_count with cap
 * once the stream has completed).
 * E_INVALID for NULL map/count pointers, n < 1, cap < 0, d_peaks NULL with
 * cap > 0, pfa outside (0, 1), or (without d_sigma2) sigma2 negative or not
 * finite. */
dsgrft_status dsgrft_detect(dsgrft_plan plan, const float *d_pmax,
                            const int32_t *d_argf, const int64_t *d_cells,
                            int64_t cc_begin, int64_t n, double sigma2,
                            const double *d_sigma2, double pfa,
                            dsgrft_peak *d_peaks, int32_t cap,
                            int32_t *d_count, dsgrft_peak *d_best,
                            int32_t *h_count, void *stream);

/* Cell-averaging CFAR along range on a reduced map (a detector beside the
 * paper's fixed LRT threshold, not in the paper): entry (cell, row r) is a
 * detection when its power exceeds alpha times the mean power of the same
 * cell's rows r' with guard < |r' - r| <= guard + train inside [0, rows);
 * the mean is a double-precision sum over r' in increasing order divided by
 * the number of such rows, and an entry without any is never a detection.
 * For exponentially distributed noise power and Nt = 2 train interior
 * training rows, alpha = Nt (P_FA^(-1/Nt) - 1) gives false-alarm probability
 * P_FA.  Map, cells, outputs, d_best and h_count (E_CAPACITY) as in
 * dsgrft_detect; guard >= 0, 1 <= train, both <= 65536, alpha finite and
 * >= 0, else E_INVALID. */
dsgrft_status dsgrft_detect_cfar(dsgrft_plan plan, const float *d_pmax,
                                 const int32_t *d_argf, const int64_t *d_cells,
                                 int64_t cc_begin, int64_t n, int32_t guard,
                                 int32_t train, double alpha, dsgrft_peak *d_peaks,
                                 int32_t cap, int32_t *d_count, dsgrft_peak *d_best,
                                 int32_t *h_count, void *stream);

/* Continuous objective for off-grid refinement (not in the paper; see the
 * oracle for the definition): for candidates theta[b] = (r0, v, a) (device
 * double [B][3]) computes Y_b (complex128) and J_b = |Y_b|^2 in FP64, and
 * stores d_saved[b] = (Y, dY/dr0, dY/dv, dY/da) as 4 complex128 for the
 * backward pass.  Orders 1 and 2 only (E_UNSUPPORTED otherwise). */
dsgrft_status dsgrft_adjoint_forward(dsgrft_plan plan, const void *d_echo,
                                     const double *d_theta, int32_t B,
                                     double *d_J, double *d_saved,
                                     void *stream);

/* Backward pass: d_grad_theta[b][p] = gJ[b] * dJ_b/dtheta_p (FP64, from the
 * saved values) and, if d_grad_echo is not NULL, d_grad_echo[m][n] =
 * sum_b gJ[b] * 2 Y_b conj(sinc(x_bm - n) exp(j phi_bm)) as complex64
 * (PyTorch's gradient convention for complex inputs), overwritten. */
dsgrft_status dsgrft_adjoint_backward(dsgrft_plan plan, const void *d_echo,
                                      const double *d_theta, int32_t B,
                                      const double *d_saved,
                                      const double *d_gJ,
                                      double *d_grad_theta, void *d_grad_echo,
                                      void *stream);

/* Off-grid peak refinement: `iters` steps of per-candidate gradient ascent
 * on J with a trust region in fine-step units (theta updated in place, final
 * J in d_J).  Each step takes the normalised gradient direction scaled by the
 * candidate's trust radius, accepts it if J does not decrease and doubles the
 * radius (capped), otherwise halves the radius.  Candidates stay inside the
 * coarse cell they started in. */
dsgrft_status dsgrft_refine(dsgrft_plan plan, const void *d_echo,
                            double *d_theta, int32_t B, int32_t iters,
                            double *d_J, void *stream);

/* Kernel timing for measurement.  Between dsgrft_profile_begin and
 * dsgrft_profile_end the plan records a HIP event pair around each launch of
 * the gather kernel (stages a1 + a2, on the plan's producer stream, where it
 * may run beside a fine search) and of the fine-search kernel (stages a3 +
 * a4, on the caller's stream) issued by dsgrft_search, for at
 * most `capacity` launches of each; later launches are not timed.  begin
 * creates the events (it is not an execution call) and resets the counters;
 * end synchronises the device, sums the event durations and destroys the
 * events.  Algorithmic work per launch: gather bytes = units x rows x M x
 * (8 read + bytes per gathered sample written); fine flops = 8 per
 * cell-pulse (one complex multiply-add), independent of the split.
 * Executed matrix work (MFMA forms; 0 for the FP32 and FFT forms): the
 * padded rows x padded table columns x padded pulses x 2 flops x the real
 * products taken per (row, column, pulse): 4 per split part, 3 for F16_3M,
 * and per conjugate-pair column 4 (F16_SYM) or 4 per split part (BF16_SYM). */
typedef struct {
  int64_t gather_launches, fine_launches;  /* timed launches               */
  double gather_ms, fine_ms;               /* summed durations            */
  double gather_bytes;                     /* algorithmic bytes, timed    */
  double fine_flops;                       /* algorithmic flops, timed    */
  double fine_cell_pulses;                 /* cells x pulses, timed       */
  double fine_mfma_flops;                  /* executed MFMA flops, timed  */
} dsgrft_profile;

dsgrft_status dsgrft_profile_begin(dsgrft_plan plan, int32_t capacity);
dsgrft_status dsgrft_profile_end(dsgrft_plan plan, dsgrft_profile *out);

/* Attainable matrix-core rate, for the roofline (a measurement aid, not part
 * of the method).  Under sustained matrix work on random data the chip runs
 * at a power-limited clock, below the one the published peak assumes.  This
 * runs a register-only loop of v_mfma_f32_32x32x16_f16 (form
 * DSGRFT_FORM_F16), _bf16 (DSGRFT_FORM_BF16) or
 * v_mfma_scale_f32_32x32x64_f8f6f4 on e4m3 operands (DSGRFT_FORM_FP8) on
 * random operands (random signs and mantissas; exponents in [2^-8, 2^1) for
 * fp16 and bf16, in [2^-1, 2^8) for e4m3 with block scales 2^-8 and 2^-7;
 * each MFMA takes another operand pair; no memory traffic) on the current
 * device, for about `ms` milliseconds after a warm-up, on the default
 * stream, and waits for it.  *h_tflops receives the executed rate (32768
 * flops per 16-bit MFMA, 131072 per e4m3 MFMA) and *h_ghz
 * the mean shader clock the workgroups read while it ran.  Allocates two
 * small device buffers for its results (it is not an execution entry
 * point).  E_INVALID for another form, NULL outputs or ms outside
 * [1, 10000]. */
dsgrft_status dsgrft_mfma_probe(dsgrft_form form, double ms, double *h_tflops, double *h_ghz);

#ifdef __cplusplus
}
#endif

#endif /* DSGRFT_H */
