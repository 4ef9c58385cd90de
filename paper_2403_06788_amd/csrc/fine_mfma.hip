// Stages a3 + a4: the fine (DFM-scale) search as a batched complex GEMM on
// MFMA with a fused |.|^2 and max/argmax epilogue.
//
// For every gathered unit u (coarse cell, and for P = 3 one fine jerk
// offset) and range row n the GFT of eq. (44) / Alg. 2 at every fine cell f of
// orders 1..min(P, 2) is
//   Y[u][f][n] = sum_m F[f][m] * G[u][n][m]            (complex)
// with F the fine phase matrix shared by all units (plan table) and G the
// gathered, de-ramped slow-time rows (stages a1 + a2).  As real MFMA products:
//   Yr = Fr Gr - Fi Gi,  Yi = Fr Gi + Fi Gr,
// all accumulated in FP32.  With both operands split into hi + lo parts the
// products taken are, by split count: 1: Fh Gh; 2: + Fl Gh; 3: + Fh Gl;
// 4: + Fl Gl.
//
// k_fine_mfma3 (below) forms the fp16 split-1 product from three real
// products per complex product instead of four; k_fine_mfma_sym takes the
// fine cells in conjugate pairs, four real products for two cells.
//
// Operand formats: fp16 and bf16 (v_mfma_f32_32x32x16, 16 pulses per K
// step, 1 KiB fragments) and OCP e4m3 (v_mfma_scale_f32_32x32x64_f8f6f4, 64
// pulses per K step, 2 KiB fragments) whose E8M0 block scales carry the
// power-of-two factors of the 8-bit encoding: 2^-8 (hi) and 2^-12 (lo) for
// the fine table, and a per-(unit, row) exponent for G.  The instruction
// takes the scale of row i's K block from lanes i and i + 32; both lanes
// carry the row's scale, so one scale per row is exact.
//
// Work decomposition: a workgroup of 2 x 2 waves computes a 128 (fine) x
// 64 WNB (row) tile of one unit; each wave a 64 x 32 WNB sub-tile as 2 x WNB
// blocks of 32 x 32 MFMAs (fine cells on the MFMA rows, range rows on its
// columns).  The wider wave tile reuses each fragment read from LDS for more
// MFMAs: the kernel is bound by LDS traffic (copies in plus fragment reads),
// not by the MFMA issue.  Accumulators live in the unified register file
// (the fp16 split-1 kernel: 222 registers, two waves per SIMD).  Operand
// fragments are stored pre-swizzled in global memory.
//
// Pipeline (one K step):
//  * operands move global -> LDS with direct LDS-DMA loads (16 bytes per
//    lane; one 1 KiB fragment half per wave and chunk row), into a ring of
//    NST stages issued NST - 1 steps ahead;
//  * each wave reads the next step's fragments from LDS into a second
//    register set while the MFMAs of the current step run, so neither the
//    copy latency nor the LDS latency sits in front of the MFMAs;
//  * one barrier per step makes the next stage (written by all waves'
//    copies) visible; slot reuse is safe because a slot is refilled only
//    after every wave has passed the barrier that follows its last read.
// Tiles are assigned XCD by XCD (workgroup ids are dealt round-robin to the 8
// XCDs), and within an XCD grouped so that concurrent tiles share fine and
// row operands in that XCD's L2.
//
// Epilogue: P = Yr^2 + Yi^2 per cell; each lane keeps the best
// (P, -fine) pair of its range row over its 32 fine cells, the two lane
// halves are merged, and one 64-bit atomicMax per (row, wave) merges
// (power bits << 32 | ~fine) into the per-(cell, row) result: the largest
// power wins and equal powers resolve to the smaller fine index, whatever the
// order of the atomics.
#include <type_traits>

#include "internal.h"

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void;

// One lane's share of an operand fragment: FR 16-byte chunks.
template <int FR>
struct Frag {
  uint4 v[FR];
};

__device__ inline uint4 xor4(uint4 a, unsigned m) {
  return make_uint4(a.x ^ m, a.y ^ m, a.z ^ m, a.w ^ m);
}

struct OpF16 {
  static constexpr int FR = 1, KSTEP = 16;
  static __device__ inline f16v mma(const Frag<1> &a, const Frag<1> &b, f16v c, int, int) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(h8, a.v[0]),
                                                  __builtin_bit_cast(h8, b.v[0]), c, 0, 0, 0);
  }
  static __device__ inline Frag<1> neg(const Frag<1> &a) { return {{xor4(a.v[0], 0x80008000u)}}; }
};

struct OpBF16 {
  static constexpr int FR = 1, KSTEP = 16;
  static __device__ inline f16v mma(const Frag<1> &a, const Frag<1> &b, f16v c, int, int) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(b8, a.v[0]),
                                                   __builtin_bit_cast(b8, b.v[0]), c, 0, 0, 0);
  }
  static __device__ inline Frag<1> neg(const Frag<1> &a) { return {{xor4(a.v[0], 0x80008000u)}}; }
};

struct OpF8 {
  static constexpr int FR = 2, KSTEP = 64;
  // sa, sb: E8M0 codes (2^(code - 127)) of the A (fine) and B (row) blocks
  static __device__ inline f16v mma(const Frag<2> &a, const Frag<2> &b, f16v c, int sa, int sb) {
    const i8v A = {(int)a.v[0].x, (int)a.v[0].y, (int)a.v[0].z, (int)a.v[0].w,
                   (int)a.v[1].x, (int)a.v[1].y, (int)a.v[1].z, (int)a.v[1].w};
    const i8v B = {(int)b.v[0].x, (int)b.v[0].y, (int)b.v[0].z, (int)b.v[0].w,
                   (int)b.v[1].x, (int)b.v[1].y, (int)b.v[1].z, (int)b.v[1].w};
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, B, c, 0, 0, 0, sa, 0, sb);
  }
  static __device__ inline Frag<2> neg(const Frag<2> &a) {
    return {{xor4(a.v[0], 0x80808080u), xor4(a.v[1], 0x80808080u)}};
  }
};

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

struct TileMap {
  int64_t u;
  int nt, ft;
};

// XCD-aware tile assignment.  Workgroup b runs on XCD b % 8; XCD x receives
// a contiguous range of tiles.  Inside a unit, tiles are visited in groups of
// GN row tiles, fine tiles major inside the group, so ~64 concurrent tiles
// of one XCD span GN row tiles x 64/GN fine tiles.
__device__ inline TileMap map_tile(int64_t bid, int64_t T, int NT, int FT, int GN) {
  int64_t q = T >> 3, r8 = T & 7, x = bid & 7, local = bid >> 3;
  int64_t tile = x * q + (x < r8 ? x : r8) + local;
  int64_t TU = (int64_t)NT * FT;
  TileMap tm;
  tm.u = tile / TU;
  int64_t rem = tile % TU;
  int64_t ng = rem / ((int64_t)GN * FT);
  int gn = NT - (int)ng * GN;
  gn = gn < GN ? gn : GN;
  int64_t idx = rem - ng * GN * FT;
  tm.ft = (int)(idx / gn);
  tm.nt = (int)(ng * GN + idx % gn);
  return tm;
}

// Product sets.  Split s (1..4) takes the first s of Fh Gh, Fl Gh, Fh Gl,
// Fl Gl; SPLIT_GLO takes Fh Gh and Fh Gl (the gathered rows split, the fine
// table not).
constexpr int SPLIT_GLO = 5;
constexpr int n_products(int split) { return split == SPLIT_GLO ? 2 : split; }
constexpr bool f_lo(int split, int s) { return split != SPLIT_GLO && (s == 1 || s == 3); }
constexpr bool g_lo(int split, int s) { return split == SPLIT_GLO ? s == 1 : s >= 2; }

// Tile shape and pipeline depth per operand format and split count.  A
// stage holds NPF planes x 4 fine fragments and NPG planes x 2 WNB row
// fragments.  Two workgroups share a CU when their rings fit in 160 KiB
// and their registers in the 512 of a SIMD lane.
template <class Op, int SPLIT>
struct Cfg {
  static constexpr int FR = Op::FR;
  static constexpr int NPF = (SPLIT >= 2 && SPLIT != SPLIT_GLO) ? 4 : 2;  // fine-table planes
  static constexpr int NPG = SPLIT >= 3 ? 4 : 2;  // gathered planes (lo from split 3, GLO)
  static constexpr int WNB = FR == 1 ? 2 : 1;
  static constexpr int NBG = 2 * WNB;             // row fragments per plane
  static constexpr int NFRAG = NPF * 4 + NPG * NBG;
  static constexpr int CH = NFRAG * FR * 64;      // 16-byte chunks per stage
  static constexpr int CPT = CH / 256;            // chunks per thread
  static constexpr int STAGE = CH * 16;
  static constexpr int NST = 4 * STAGE <= 80 * 1024 ? 4 : 3;
  // two workgroups per CU also need two register sets: split 1 only
  static constexpr int MINB = (SPLIT == 1 && NST * STAGE <= 80 * 1024) ? 2 : 1;
  static_assert(CH % 256 == 0, "stage must split evenly over 256 threads");
  static_assert(NST * STAGE <= 160 * 1024, "ring exceeds LDS");
};

// Wait until at most `ahead` stages of this wave's copies are in flight,
// then barrier: afterwards every wave's copies of the stage are in LDS.  The
// barrier carries no LDS fence: the slot refilled after it was last read two
// steps earlier, by reads whose results the previous step's MFMAs consumed,
// so no LDS read of it can still be in flight (needs NST >= 3).  Wait and
// barrier share one asm statement with a memory clobber so that no LDS read
// is hoisted above the barrier.
template <int CPT>
__device__ inline void wait_copies_barrier(int ahead) {
  __builtin_amdgcn_sched_barrier(0);
  if (ahead >= 2) {
    asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(2 * CPT) : "memory");
  } else if (ahead == 1) {
    asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(CPT) : "memory");
  } else {
    asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
  }
}

// Instruction order inside one K step: the next step's LDS reads first, then
// the MFMAs of this step.
template <class CF, int SPLIT>
__device__ inline void order_step() {
  __builtin_amdgcn_sched_group_barrier(0x100, (CF::NPF * 2 + CF::NPG * CF::WNB) * CF::FR, 0);
  __builtin_amdgcn_sched_group_barrier(0x008, n_products(SPLIT) * 8 * CF::WNB, 0);
}

template <class CF>
__device__ inline void read_frags(const uint4 *__restrict__ slot, int wf, int wn,
                                  int lane, Frag<CF::FR> (&a)[CF::NPF][2],
                                  Frag<CF::FR> (&b)[CF::NPG][CF::WNB]) {
  constexpr int FR = CF::FR;
#pragma unroll
  for (int p = 0; p < CF::NPF; ++p)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int h = 0; h < FR; ++h)
        a[p][i].v[h] = slot[((p * 4 + wf * 2 + i) * FR + h) * 64 + lane];
#pragma unroll
  for (int p = 0; p < CF::NPG; ++p)
#pragma unroll
    for (int j = 0; j < CF::WNB; ++j)
#pragma unroll
      for (int h = 0; h < FR; ++h)
        b[p][j].v[h] =
            slot[((CF::NPF * 4 + p * CF::NBG + wn * CF::WNB + j) * FR + h) * 64 + lane];
}

// Empty asm "redefining" a fragment set: MFMAs that consume the set cannot
// be scheduled above this point.  Placed after each step's barrier, it keeps
// the next step's MFMAs (and the waits for their LDS reads) out of the
// current step.
template <int FR>
__device__ inline void pin1(Frag<FR> &f) {
#pragma unroll
  for (int h = 0; h < FR; ++h)
    asm volatile("" : "+v"(f.v[h].x), "+v"(f.v[h].y), "+v"(f.v[h].z), "+v"(f.v[h].w));
}

template <class CF>
__device__ inline void pin(Frag<CF::FR> (&a)[CF::NPF][2], Frag<CF::FR> (&b)[CF::NPG][CF::WNB]) {
#pragma unroll
  for (int p = 0; p < CF::NPF; ++p)
#pragma unroll
    for (int i = 0; i < 2; ++i) pin1<CF::FR>(a[p][i]);
#pragma unroll
  for (int p = 0; p < CF::NPG; ++p)
#pragma unroll
    for (int j = 0; j < CF::WNB; ++j) pin1<CF::FR>(b[p][j]);
}

// sa[0/1]: fine-table hi/lo scale codes; sb[0/1][j]: row block j's hi/lo.
template <class Op, class CF, int SPLIT>
__device__ inline void mma_step(const Frag<CF::FR> (&a)[CF::NPF][2],
                                const Frag<CF::FR> (&b)[CF::NPG][CF::WNB],
                                f16v (&accR)[2][CF::WNB], f16v (&accI)[2][CF::WNB],
                                const int (&sa)[2], const int (&sb)[2][CF::WNB]) {
#pragma unroll
  for (int s = 0; s < n_products(SPLIT); ++s) {
    const int la = f_lo(SPLIT, s) ? 1 : 0;  // fine table lo
    const int lb = g_lo(SPLIT, s) ? 1 : 0;  // gathered lo
    const int pa = 2 * la, pb = 2 * lb;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const Frag<CF::FR> nfi = Op::neg(a[pa + 1][i]);
#pragma unroll
      for (int j = 0; j < CF::WNB; ++j) {
        const int x = sa[la], y = sb[lb][j];
        accR[i][j] = Op::mma(a[pa][i], b[pb][j], accR[i][j], x, y);
        accR[i][j] = Op::mma(nfi, b[pb + 1][j], accR[i][j], x, y);
        accI[i][j] = Op::mma(a[pa][i], b[pb + 1][j], accI[i][j], x, y);
        accI[i][j] = Op::mma(a[pa + 1][i], b[pb][j], accI[i][j], x, y);
      }
    }
  }
}

// F, G: operand fragments; KS: K steps (Mp / Op::KSTEP); gsc: per-(unit,
// row) scale codes of G (8-bit form only); fsc: the fine table's hi scale
// code (lo is 4 below).
template <class Op, int SPLIT>
__global__ __launch_bounds__(256, (Cfg<Op, SPLIT>::MINB)) void k_fine_mfma(
    const uint4 *__restrict__ F, const uint4 *__restrict__ G,
    const int32_t *__restrict__ gsc, int fsc, const int32_t *__restrict__ gshift,
    unsigned long long *__restrict__ packed, float *__restrict__ full, int FB,
    int NB, int KS, int rows_p, int64_t nunits, int64_t unit0, int R3, int C,
    int rows, int GN) {
  using CF = Cfg<Op, SPLIT>;
  constexpr int FR = CF::FR, NPF = CF::NPF, NPG = CF::NPG, NST = CF::NST;
  constexpr int CH = CF::CH, CPT = CF::CPT, WNB = CF::WNB, NBG = CF::NBG;
  __shared__ uint4 lds[NST][CH];

  const int NT = NB / NBG, FT = FB >> 2;
  const TileMap tm = map_tile(blockIdx.x, nunits * NT * FT, NT, FT, GN);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wf = wave & 1, wn = wave >> 1;
  const int wbase = tid & ~63;

  // block scales (8-bit form); the asm consumes the loaded values here so
  // that their wait is not placed after the first copies are in flight
  int sa[2] = {fsc, fsc - 4};
  int sb[2][WNB];
#pragma unroll
  for (int j = 0; j < WNB; ++j) {
    sb[0][j] = 0;
    if (gsc != nullptr) {
      const int n = (tm.nt * NBG + wn * WNB + j) * 32 + (lane & 31);
      sb[0][j] = gsc[tm.u * rows_p + n];
      asm volatile("" : "+v"(sb[0][j]));
    }
    sb[1][j] = sb[0][j] - 4;
  }

  // Global source of this thread's chunks (16-byte units).  Chunk c of a
  // stage: lane c % 64, half (c / 64) % FR, fragment (c / 64) / FR: fine
  // fragments first (plane-major, 4 per plane), then row fragments (NBG per
  // plane).
  const uint4 *src[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int c = tid + 256 * j;
    const int ln = c & 63, h = (c >> 6) % FR, fi = (c >> 6) / FR;
    if (fi < NPF * 4) {
      const int plane = fi >> 2, blk = fi & 3;
      src[j] = F + (((int64_t)plane * FB + tm.ft * 4 + blk) * KS) * (FR * 64) + h * 64 + ln;
    } else {
      const int gi = fi - NPF * 4, plane = gi / NBG, blk = gi % NBG;
      src[j] = G + (((tm.u * NPG + plane) * NB + tm.nt * NBG + blk) * (int64_t)KS) * (FR * 64) +
               h * 64 + ln;
    }
  }
  // Copy K step `stage` into its ring slot: global_load_lds_dwordx4 writes
  // lane l's 16 bytes to LDS at M0 + 16 l.  It is issued from inline
  // assembly so that the compiler, which cannot tell the ring slots apart,
  // does not put a wait for every copy in flight in front of each LDS read;
  // completion is awaited explicitly (wait_copies) before the barrier that
  // publishes a stage.  The instruction has no register results; M0 is saved
  // and restored around it.
  auto issue = [&](int stage) {
    uint4 *dst = lds[stage % NST];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const unsigned la = __builtin_amdgcn_readfirstlane(
          (unsigned)(size_t)(lds_void *)&dst[wbase + 256 * j]);
      const uint4 *g = src[j] + (int64_t)stage * (FR * 64);
      unsigned saved_m0;
      asm volatile(
          "s_mov_b32 %0, m0\n\t"
          "s_mov_b32 m0, %1\n\t"
          "s_nop 0\n\t"
          "global_load_lds_dwordx4 %2, off\n\t"
          "s_nop 0\n\t"
          "s_mov_b32 m0, %0"
          : "=&s"(saved_m0)
          : "s"(la), "v"(g)
          : "memory");
    }
  };

  f16v accR[2][WNB], accI[2][WNB];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < WNB; ++j) {
      accR[i][j] = f16v{};
      accI[i][j] = f16v{};
    }

  const int nkt = KS;
  // prologue: stages 0 .. NST-2 in flight, stage 0 visible, its fragments read
#pragma unroll
  for (int s = 0; s < NST - 1; ++s)
    if (s < nkt) issue(s);
  wait_copies_barrier<CPT>((nkt - 1 < NST - 2) ? nkt - 1 : NST - 2);
  Frag<FR> a0[NPF][2], b0[NPG][WNB], a1[NPF][2], b1[NPG][WNB];
  read_frags<CF>(lds[0], wf, wn, lane, a0, b0);

  // One K step: make stage kt+1 visible, read its fragments into (an, bn),
  // refill the slot freed one step ago, then the MFMAs of step kt.
#define DS_STEP(KT, AC, BC, AN, BN)                                              \
  do {                                                                         \
    const int kt_ = (KT);                                                      \
    if (kt_ + 1 < nkt) {                                                       \
      const int last = (nkt - 1 < kt_ + NST - 2) ? nkt - 1 : kt_ + NST - 2;    \
      wait_copies_barrier<CPT>(last - (kt_ + 1));                              \
      pin<CF>(AC, BC);                                                         \
      read_frags<CF>(lds[(kt_ + 1) % NST], wf, wn, lane, AN, BN);              \
      if (kt_ + NST - 1 < nkt) issue(kt_ + NST - 1);                           \
    }                                                                          \
    mma_step<Op, CF, SPLIT>(AC, BC, accR, accI, sa, sb);                       \
  } while (0)

  // Steady state, branch-free: every step waits for the same number of
  // copies in flight and refills a slot.
#define DS_STEADY(KT, AC, BC, AN, BN)                                          \
  do {                                                                         \
    const int kt_ = (KT);                                                      \
    wait_copies_barrier<CPT>(NST - 3);                                         \
    pin<CF>(AC, BC);                                                           \
    read_frags<CF>(lds[(kt_ + 1) % NST], wf, wn, lane, AN, BN);                \
    issue(kt_ + NST - 1);                                                      \
    mma_step<Op, CF, SPLIT>(AC, BC, accR, accI, sa, sb);                       \
    order_step<CF, SPLIT>();                                                   \
  } while (0)
  int kt = 0;
  for (; kt + NST < nkt; kt += 2) {
    DS_STEADY(kt, a0, b0, a1, b1);
    DS_STEADY(kt + 1, a1, b1, a0, b0);
  }
#undef DS_STEADY
  for (; kt < nkt; kt += 2) {
    DS_STEP(kt, a0, b0, a1, b1);
    if (kt + 1 < nkt) DS_STEP(kt + 1, a1, b1, a0, b0);
  }
#undef DS_STEP

  // ---- epilogue: |Y|^2, best fine cell per row, merge -----------------
  // (fp16 rows carry the echo shift 2^sh: the power is scaled by 2^-2sh)
  const int psh = gshift != nullptr ? -2 * gshift[1] : 0;
  const int64_t ug = unit0 + tm.u;
  const int64_t cpos = ug / R3;
  const unsigned fbase = (unsigned)((ug % R3) * C);
#pragma unroll
  for (int j = 0; j < WNB; ++j) {
    const int n = (tm.nt * NBG + wn * WNB + j) * 32 + (lane & 31);
    unsigned long long best = 0ull;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int fb0 = (tm.ft * 4 + wf * 2 + i) * 32 + 4 * (lane >> 5);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = fb0 + 8 * (r >> 2) + (r & 3);
        const float yr = accR[i][j][r], yi = accI[i][j][r];
        const float pw = ldexpf(yr * yr + yi * yi, psh);
        if (f < C) {
          const unsigned ff = fbase + (unsigned)f;
          const unsigned long long key =
              ((unsigned long long)__float_as_uint(pw) << 32) | (0xffffffffu - ff);
          best = umax64(best, key);
          if (full != nullptr && n < rows)
            full[(cpos * rows + n) * (int64_t)(C * R3) + ff] = pw;
        }
      }
    }
    best = umax64(best, shfl_xor64(best, 32));
    if (lane < 32 && n < rows) atomicMax(&packed[cpos * rows + n], best);
  }
}

// The fp16 search with three real products per complex product (Gauss's
// form of the complex multiplication):
//   P1 = Fr Gr,  P2 = Fi Gi,  P3 = (Fr + Fi)(Gr + Gi),
//   Yr = P1 - P2,  Yi = P3 - P1 - P2,
// 12 MFMAs per K step and wave instead of 16, same algorithmic result.  The
// operand sums are formed in registers from the fp16 hi planes
// (v_pk_add_f16, round to nearest even), so the tables and the gather are
// those of the fp16 split-1 form; their rounding enters Yi only.  Under
// sustained random-operand MFMA load the chip runs at a power-limited
// clock, so a quarter fewer matrix products is a quarter less of the energy
// that sets it.
//
// Tile as k_fine_mfma<OpF16, 1>: 128 fine x 128 rows per workgroup, 64 x 64
// per wave (2 x 2 blocks of 32x32x16); four LDS slots of 16 KiB filled by
// LDS-DMA a pair of K steps ahead, one barrier per pair.  The three
// accumulator sets take 192 registers, so there is no second fragment set:
// each step reads its own fragments, and the other workgroup's wave on the
// same SIMD (two per CU) issues its MFMAs meanwhile.
__device__ inline uint4 add_h8(uint4 a, uint4 b) {
  return __builtin_bit_cast(uint4, __builtin_bit_cast(h8, a) + __builtin_bit_cast(h8, b));
}

__global__ __launch_bounds__(256, 2) void k_fine_mfma3(
    const uint4 *__restrict__ F, const uint4 *__restrict__ G, const int32_t *__restrict__ gshift,
    unsigned long long *__restrict__ packed, float *__restrict__ full, int FB,
    int NB, int KS, int64_t nunits, int64_t unit0, int R3, int C, int rows, int GN) {
  constexpr int NST = 4, NBG = 4;
  constexpr int CH = 16 * 64, CPT = CH / 256;  // 16 fragments per stage
  __shared__ uint4 lds[NST][CH];

  const int NT = NB / NBG, FT = FB >> 2;
  const TileMap tm = map_tile(blockIdx.x, nunits * NT * FT, NT, FT, GN);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wf = wave & 1, wn = wave >> 1;
  const int wbase = tid & ~63;

  // Chunk c of a stage: lane c % 64, fragment c / 64: fine (re 0-3, im 4-7),
  // then rows (re 8-11, im 12-15).
  const uint4 *src[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int c = tid + 256 * j;
    const int ln = c & 63, fi = c >> 6;
    if (fi < 8) {
      const int plane = fi >> 2, blk = fi & 3;
      src[j] = F + (((int64_t)plane * FB + tm.ft * 4 + blk) * KS) * 64 + ln;
    } else {
      const int plane = (fi - 8) >> 2, blk = fi & 3;
      src[j] = G + (((tm.u * 2 + plane) * NB + tm.nt * NBG + blk) * (int64_t)KS) * 64 + ln;
    }
  }
  auto issue = [&](int stage) {
    uint4 *dst = lds[stage % NST];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const unsigned la = __builtin_amdgcn_readfirstlane(
          (unsigned)(size_t)(lds_void *)&dst[wbase + 256 * j]);
      const uint4 *g = src[j] + (int64_t)stage * 64;
      unsigned saved_m0;
      asm volatile(
          "s_mov_b32 %0, m0\n\t"
          "s_mov_b32 m0, %1\n\t"
          "s_nop 0\n\t"
          "global_load_lds_dwordx4 %2, off\n\t"
          "s_nop 0\n\t"
          "s_mov_b32 m0, %0"
          : "=&s"(saved_m0)
          : "s"(la), "v"(g)
          : "memory");
    }
  };

  f16v acc[3][2][2];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[q][i][j] = f16v{};

  // One K step: read the step's fragments, P1 and P2, the operand sums, P3.
  auto step = [&](int kt) {
    const uint4 *slot = lds[kt % NST];
    uint4 fr[2], fi[2], gr[2], gi[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) fr[i] = slot[(wf * 2 + i) * 64 + lane];
#pragma unroll
    for (int j = 0; j < 2; ++j) gr[j] = slot[(8 + wn * 2 + j) * 64 + lane];
#pragma unroll
    for (int i = 0; i < 2; ++i) fi[i] = slot[(4 + wf * 2 + i) * 64 + lane];
#pragma unroll
    for (int j = 0; j < 2; ++j) gi[j] = slot[(12 + wn * 2 + j) * 64 + lane];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[0][i][j] = OpF16::mma({{fr[i]}}, {{gr[j]}}, acc[0][i][j], 0, 0);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[1][i][j] = OpF16::mma({{fi[i]}}, {{gi[j]}}, acc[1][i][j], 0, 0);
    uint4 fs[2], gs[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) fs[i] = add_h8(fr[i], fi[i]);
#pragma unroll
    for (int j = 0; j < 2; ++j) gs[j] = add_h8(gr[j], gi[j]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[2][i][j] = OpF16::mma({{fs[i]}}, {{gs[j]}}, acc[2][i][j], 0, 0);
  };

  // Steps go in pairs (KS is a multiple of 4), one barrier per pair: the
  // pair (kt, kt + 1) waits for its own copies, and the next pair is copied
  // into the slots of the previous one, which every wave finished before
  // this barrier.
  const int nkt = KS;
  issue(0);
  issue(1);
  for (int kt = 0; kt < nkt; kt += 2) {
    wait_copies_barrier<CPT>(0);
    if (kt + 2 < nkt) {
      issue(kt + 2);
      issue(kt + 3);
    }
    step(kt);
    step(kt + 1);
  }

  // ---- epilogue as in k_fine_mfma ----------------------------------------
  const int psh = -2 * gshift[1];
  const int64_t ug = unit0 + tm.u;
  const int64_t cpos = ug / R3;
  const unsigned fbase = (unsigned)((ug % R3) * C);
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int n = (tm.nt * NBG + wn * 2 + j) * 32 + (lane & 31);
    unsigned long long best = 0ull;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int fb0 = (tm.ft * 4 + wf * 2 + i) * 32 + 4 * (lane >> 5);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = fb0 + 8 * (r >> 2) + (r & 3);
        const float p1 = acc[0][i][j][r], p2 = acc[1][i][j][r], p3 = acc[2][i][j][r];
        const float yr = p1 - p2, yi = p3 - p1 - p2;
        const float pw = ldexpf(yr * yr + yi * yi, psh);
        if (f < C) {
          const unsigned ff = fbase + (unsigned)f;
          const unsigned long long key =
              ((unsigned long long)__float_as_uint(pw) << 32) | (0xffffffffu - ff);
          best = umax64(best, key);
          if (full != nullptr && n < rows)
            full[(cpos * rows + n) * (int64_t)(C * R3) + ff] = pw;
        }
      }
    }
    best = umax64(best, shfl_xor64(best, 32));
    if (lane < 32 && n < rows) atomicMax(&packed[cpos * rows + n], best);
  }
}

// The search over conjugate pairs of fine cells.  A fine cell's offsets d
// from the coarse centre are symmetric about it (R/2 on either side, for
// even R one more on the negative side) and its phase is linear in d, so the
// cell at -d has the conjugate fine phasor of the cell at +d.  With the four
// real products of the +d column, Prr = Fr Gr, Pii = Fi Gi, Pri = Fr Gi,
// Pir = Fi Gr:
//   Y(+d) = (Prr - Pii) + j (Pri + Pir),
//   Y(-d) = (Prr + Pii) + j (Pri - Pir),
// the same operands, products and FP32 sums as the four-product form, but
// half the columns: 8 MFMAs per K step and wave cover 64 cells x 64 rows
// (12 in k_fine_mfma3, 16 in k_fine_mfma<f16, 1>).  The table F holds one
// column per pair, plus the cells without a partner (an offset of -R/2 for
// even R, and the centre), ordered by cols[c] (the +d cell) and
// cols[ncols + c] (the -d cell, -1 if none); padding columns are zero.
//
// The bf16 forms add split parts; the four products are linear in both
// operands, so every part accumulates into the same four sets:
//   NPF = 2, NPG = 4: Fh Gh + Fh Gl (the gathered rows split into hi + lo),
//     16 MFMAs per K step and wave for 64 cells x 64 rows (32 in
//     k_fine_mfma<bf16, rows split>);
//   NPF = 4, NPG = 4: + Fl Gh (the table's lo part; Fl(-d) is the conjugate
//     of Fl(+d) as well, rounding being symmetric), 24 MFMAs (48 in
//     k_fine_mfma<bf16, 3>).
// Within a step, every product part runs over all eight accumulators before
// the next part.
//
// Tile: 64 columns x 128 rows per workgroup, 32 columns x 64 rows per wave (1
// x 2 blocks of 32x32x16), four accumulator sets (128 registers; 167 in all
// for the fp16 form).  Stages of 2 NPF column and 4 NPG row fragments (12, 20
// or 24 KiB) are filled by LDS-DMA into a ring: four slots a pair of K steps
// ahead with one barrier per pair (as in k_fine_mfma3) when the ring fits
// beside the other workgroups of the CU, else three slots two steps ahead
// with one barrier per step.  Workgroups per CU: three (fp16, 144 KiB of
// LDS, three waves per SIMD) or two (bf16; 160 and 144 KiB).  Tiles are
// grouped by four row tiles (GN = 4; for the fp16 form, 8 and 16 were 3% and
// 9% slower, 2 and 6 within 1%).
template <int NPF, int NPG>
struct SymCfg {
  static constexpr int NFR = 2 * NPF + 4 * NPG;    // fragments per stage
  static constexpr int CH = NFR * 64, CPT = CH / 256;
  static constexpr int WG = NPG == 2 ? 3 : 2;      // workgroups per CU
  static constexpr int NST = WG * 4 * CH * 16 <= 160 * 1024 ? 4 : 3;
  static_assert(CH % 256 == 0, "stage must split evenly over 256 threads");
  static_assert(WG * NST * CH * 16 <= 160 * 1024, "rings exceed LDS");
};

template <class Op, int NPF, int NPG>
__global__ __launch_bounds__(256, (SymCfg<NPF, NPG>::WG)) void k_fine_mfma_sym(
    const uint4 *__restrict__ F, const uint4 *__restrict__ G,
    const int32_t *__restrict__ cols, const int32_t *__restrict__ gshift,
    unsigned long long *__restrict__ packed, float *__restrict__ full, int FBs, int NB,
    int KS, int64_t nunits, int64_t unit0, int R3, int C, int rows, int GN) {
  using SC = SymCfg<NPF, NPG>;
  constexpr int NST = SC::NST, CH = SC::CH, CPT = SC::CPT;
  constexpr int NBG = 4, NFB = 2;  // row / column blocks per tile
  __shared__ uint4 lds[NST][CH];

  const int NT = NB / NBG, FT = FBs / NFB;
  const TileMap tm = map_tile(blockIdx.x, nunits * NT * FT, NT, FT, GN);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wf = wave & 1, wn = wave >> 1;
  const int wbase = tid & ~63;

  // Chunk c of a stage: lane c % 64, fragment c / 64: columns, NFB per plane
  // (re_hi, im_hi[, re_lo, im_lo]), then rows, NBG per plane (re_hi,
  // im_hi[, re_lo, im_lo]).
  const uint4 *src[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int c = tid + 256 * j;
    const int ln = c & 63, fi = c >> 6;
    if (fi < NFB * NPF) {
      const int plane = fi / NFB, blk = fi % NFB;
      src[j] = F + (((int64_t)plane * FBs + tm.ft * NFB + blk) * KS) * 64 + ln;
    } else {
      const int plane = (fi - NFB * NPF) / NBG, blk = (fi - NFB * NPF) % NBG;
      src[j] = G + (((tm.u * NPG + plane) * NB + tm.nt * NBG + blk) * (int64_t)KS) * 64 + ln;
    }
  }
  auto issue = [&](int stage) {
    uint4 *dst = lds[stage % NST];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const unsigned la = __builtin_amdgcn_readfirstlane(
          (unsigned)(size_t)(lds_void *)&dst[wbase + 256 * j]);
      const uint4 *g = src[j] + (int64_t)stage * 64;
      unsigned saved_m0;
      asm volatile(
          "s_mov_b32 %0, m0\n\t"
          "s_mov_b32 m0, %1\n\t"
          "s_nop 0\n\t"
          "global_load_lds_dwordx4 %2, off\n\t"
          "s_nop 0\n\t"
          "s_mov_b32 m0, %0"
          : "=&s"(saved_m0)
          : "s"(la), "v"(g)
          : "memory");
    }
  };

  f16v acc[4][2];  // Prr, Pii, Pri, Pir per row block
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[q][j] = f16v{};

  // One product part: fr/fi a column fragment pair, gr/gi the row fragments.
  auto part = [&](const Frag<1> &fr, const Frag<1> &fi, const Frag<1> (&gr)[2],
                  const Frag<1> (&gi)[2]) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc[0][j] = Op::mma(fr, gr[j], acc[0][j], 0, 0);
      acc[1][j] = Op::mma(fi, gi[j], acc[1][j], 0, 0);
      acc[2][j] = Op::mma(fr, gi[j], acc[2][j], 0, 0);
      acc[3][j] = Op::mma(fi, gr[j], acc[3][j], 0, 0);
    }
  };
  auto step = [&](int kt) {
    const uint4 *slot = lds[kt % NST];
    Frag<1> f[NPF / 2][2], g[NPG / 2][2][2];  // [hi/lo][re/im]([row block])
#pragma unroll
    for (int h = 0; h < NPF / 2; ++h)
#pragma unroll
      for (int c = 0; c < 2; ++c) f[h][c] = {{slot[((2 * h + c) * NFB + wf) * 64 + lane]}};
#pragma unroll
    for (int h = 0; h < NPG / 2; ++h)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          g[h][c][j] = {{slot[(NFB * NPF + (2 * h + c) * NBG + wn * 2 + j) * 64 + lane]}};
    part(f[0][0], f[0][1], g[0][0], g[0][1]);  // Fh Gh
    if (NPG == 4) part(f[0][0], f[0][1], g[NPG / 2 - 1][0], g[NPG / 2 - 1][1]);  // Fh Gl
    if (NPF == 4) part(f[NPF / 2 - 1][0], f[NPF / 2 - 1][1], g[0][0], g[0][1]);  // Fl Gh
  };

  const int nkt = KS;
  if (NST == 4) {
    issue(0);
    issue(1);
    for (int kt = 0; kt < nkt; kt += 2) {
      wait_copies_barrier<CPT>(0);
      if (kt + 2 < nkt) {
        issue(kt + 2);
        issue(kt + 3);
      }
      step(kt);
      step(kt + 1);
    }
  } else {
    // three slots: step kt's stage is awaited with step kt + 1's in flight;
    // the slot refilled after the barrier was last read in step kt - 1,
    // which every wave finished before it
    issue(0);
    if (nkt > 1) issue(1);
    for (int kt = 0; kt < nkt; ++kt) {
      wait_copies_barrier<CPT>(kt + 1 < nkt ? 1 : 0);
      if (kt + 2 < nkt) issue(kt + 2);
      step(kt);
    }
  }

  // ---- epilogue: both cells of each column ---------------------------------
  const int psh = gshift != nullptr ? -2 * gshift[1] : 0;
  const int64_t ug = unit0 + tm.u;
  const int64_t cpos = ug / R3;
  const unsigned fbase = (unsigned)((ug % R3) * C);
  const int ncols = FBs * 32;
  const int cb0 = (tm.ft * NFB + wf) * 32 + 4 * (lane >> 5);
  unsigned long long best[2] = {0ull, 0ull};
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int col = cb0 + 8 * (r >> 2) + (r & 3);
    const int fp = cols[col], fm = cols[ncols + col];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = (tm.nt * NBG + wn * 2 + j) * 32 + (lane & 31);
      const float prr = acc[0][j][r], pii = acc[1][j][r];
      const float pri = acc[2][j][r], pir = acc[3][j][r];
      const float ar = prr - pii, ai = pri + pir;  // +d
      const float br = prr + pii, bi = pri - pir;  // -d
      const float pa = ldexpf(ar * ar + ai * ai, psh), pb = ldexpf(br * br + bi * bi, psh);
      if (fp >= 0) {
        const unsigned ff = fbase + (unsigned)fp;
        best[j] = umax64(best[j], ((unsigned long long)__float_as_uint(pa) << 32) | (0xffffffffu - ff));
        if (full != nullptr && n < rows) full[(cpos * rows + n) * (int64_t)(C * R3) + ff] = pa;
      }
      if (fm >= 0) {
        const unsigned ff = fbase + (unsigned)fm;
        best[j] = umax64(best[j], ((unsigned long long)__float_as_uint(pb) << 32) | (0xffffffffu - ff));
        if (full != nullptr && n < rows) full[(cpos * rows + n) * (int64_t)(C * R3) + ff] = pb;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int n = (tm.nt * NBG + wn * 2 + j) * 32 + (lane & 31);
    const unsigned long long b = umax64(best[j], shfl_xor64(best[j], 32));
    if (lane < 32 && n < rows) atomicMax(&packed[cpos * rows + n], b);
  }
}


// The e4m3 form over conjugate pairs (split 3: Fh Gh + Fl Gh + Fh Gl;
// split 4: + Fl Gl), every part into the same four real products of a pair
// with the block scales of the unpaired e4m3 form (fine table 2^-8 / 2^-12,
// one code per gathered row and its lo part 2^-4 below).  Tile as
// k_fine_mfma_sym (64 pair columns x 128 rows) with 64-pulse K steps; a stage
// holds 4 planes x 2 column and 4 planes x 4 row fragments of 2 KiB (48 KiB),
// so a three-slot ring (144 KiB) leaves one workgroup per CU.  Eight waves,
// one column block x one row block each (64 accumulator registers, 141 in
// all), make two waves per SIMD: the MFMAs of one cover the fragment reads of
// the other, which a single wave per SIMD with two register sets (two row
// blocks per wave, ~460 registers) could not do as well (4.7 ms against
// 3.6 ms per launch at M = 1024).  The ring is filled two steps ahead.
template <int SPLIT>
__global__ __launch_bounds__(512, 1) void k_fine_mfma_sym8(
    const uint4 *__restrict__ F, const uint4 *__restrict__ G,
    const int32_t *__restrict__ gsc, int fsc, const int32_t *__restrict__ cols,
    unsigned long long *__restrict__ packed, float *__restrict__ full, int FBs, int NB,
    int KS, int rows_p, int64_t nunits, int64_t unit0, int R3, int C, int rows, int GN) {
  using Op = OpF8;
  constexpr int FR = 2, NP = 4, NBG = 4, NFB = 2, NST = 3;
  constexpr int NTH = 64 * NFB * NBG;             // one wave per column x row block
  constexpr int NFR = NP * NFB + NP * NBG;        // 24 fragments per stage
  constexpr int CH = NFR * FR * 64, CPT = CH / NTH;  // 3072 chunks, 6 per thread
  static_assert(CH % NTH == 0, "stage must split evenly over the workgroup");
  __shared__ uint4 lds[NST][CH];

  const int NT = NB / NBG, FT = FBs / NFB;
  const TileMap tm = map_tile(blockIdx.x, nunits * NT * FT, NT, FT, GN);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wf = wave & 1, wn = wave >> 1;
  const int wbase = tid & ~63;

  // this lane's row and its scale codes (hi; lo is 4 below)
  const int n = (tm.nt * NBG + wn) * 32 + (lane & 31);
  int sbh = gsc[tm.u * rows_p + n];
  asm volatile("" : "+v"(sbh));
  const int sb[2] = {sbh, sbh - 4};
  const int sa[2] = {fsc, fsc - 4};

  // chunk c of a stage: lane c % 64, half (c / 64) % 2, fragment (c / 64) / 2:
  // column fragments first (plane-major, NFB per plane), then row fragments
  // (NBG per plane)
  const uint4 *src[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int c = tid + NTH * j;
    const int ln = c & 63, h = (c >> 6) % FR, fi = (c >> 6) / FR;
    if (fi < NP * NFB) {
      const int plane = fi / NFB, blk = fi % NFB;
      src[j] = F + (((int64_t)plane * FBs + tm.ft * NFB + blk) * KS) * (FR * 64) + h * 64 + ln;
    } else {
      const int gi = fi - NP * NFB, plane = gi / NBG, blk = gi % NBG;
      src[j] = G + (((tm.u * NP + plane) * NB + tm.nt * NBG + blk) * (int64_t)KS) * (FR * 64) +
               h * 64 + ln;
    }
  }
  auto issue = [&](int stage) {
    uint4 *dst = lds[stage % NST];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      const unsigned la = __builtin_amdgcn_readfirstlane(
          (unsigned)(size_t)(lds_void *)&dst[wbase + NTH * j]);
      const uint4 *g = src[j] + (int64_t)stage * (FR * 64);
      unsigned saved_m0;
      asm volatile(
          "s_mov_b32 %0, m0\n\t"
          "s_mov_b32 m0, %1\n\t"
          "s_nop 0\n\t"
          "global_load_lds_dwordx4 %2, off\n\t"
          "s_nop 0\n\t"
          "s_mov_b32 m0, %0"
          : "=&s"(saved_m0)
          : "s"(la), "v"(g)
          : "memory");
    }
  };

  f16v acc[4] = {};  // Prr, Pii, Pri, Pir

  // fragments of one K step: f[plane] (re_hi, im_hi, re_lo, im_lo) of the
  // wave's column block, g[plane] of its row block
  Frag<2> f[NP], g[NP];
  auto rd = [&](int kt) {
    const uint4 *slot = lds[kt % NST];
#pragma unroll
    for (int pl = 0; pl < NP; ++pl)
#pragma unroll
      for (int h = 0; h < FR; ++h) {
        f[pl].v[h] = slot[((pl * NFB + wf) * FR + h) * 64 + lane];
        g[pl].v[h] = slot[((NP * NFB + pl * NBG + wn) * FR + h) * 64 + lane];
      }
  };
  // one product part: fine planes (pf, pf + 1) at scale la, row planes
  // (pg, pg + 1) at scale lb
  auto part = [&](int pf, int pg, int la, int lb) {
    const int A = sa[la], B = sb[lb];
    acc[0] = Op::mma(f[pf], g[pg], acc[0], A, B);
    acc[1] = Op::mma(f[pf + 1], g[pg + 1], acc[1], A, B);
    acc[2] = Op::mma(f[pf], g[pg + 1], acc[2], A, B);
    acc[3] = Op::mma(f[pf + 1], g[pg], acc[3], A, B);
  };
  auto mm = [&]() {
    part(0, 0, 0, 0);                 // Fh Gh
    part(2, 0, 1, 0);                 // Fl Gh
    part(0, 2, 0, 1);                 // Fh Gl
    if (SPLIT == 4) part(2, 2, 1, 1);  // Fl Gl
  };

  // three slots, stages k + 1 and k + 2 in flight during step k: the slot
  // that stage k + 2 fills held stage k - 1, which every wave read (and
  // waited for) before the barrier of step k
  const int nkt = KS;
  issue(0);
  if (nkt > 1) issue(1);
  int kt = 0;
  for (; kt + 2 < nkt; ++kt) {
    asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(CPT) : "memory");
    issue(kt + 2);
    rd(kt);
    mm();
  }
  for (; kt < nkt; ++kt) {
    if (kt + 1 < nkt)
      asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(CPT) : "memory");
    else
      asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    rd(kt);
    mm();
  }
  // ---- epilogue: both cells of each column ---------------------------------
  const int64_t ug = unit0 + tm.u;
  const int64_t cpos = ug / R3;
  const unsigned fbase = (unsigned)((ug % R3) * C);
  const int ncols = FBs * 32;
  const int cb0 = (tm.ft * NFB + wf) * 32 + 4 * (lane >> 5);
  unsigned long long best = 0ull;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int col = cb0 + 8 * (r >> 2) + (r & 3);
    const int fp = cols[col], fm = cols[ncols + col];
    const float prr = acc[0][r], pii = acc[1][r];
    const float pri = acc[2][r], pir = acc[3][r];
    const float ar = prr - pii, ai = pri + pir;  // +d
    const float br = prr + pii, bi = pri - pir;  // -d
    const float pa = ar * ar + ai * ai, pb = br * br + bi * bi;
    if (fp >= 0) {
      const unsigned ff = fbase + (unsigned)fp;
      best = umax64(best, ((unsigned long long)__float_as_uint(pa) << 32) | (0xffffffffu - ff));
      if (full != nullptr && n < rows) full[(cpos * rows + n) * (int64_t)(C * R3) + ff] = pa;
    }
    if (fm >= 0) {
      const unsigned ff = fbase + (unsigned)fm;
      best = umax64(best, ((unsigned long long)__float_as_uint(pb) << 32) | (0xffffffffu - ff));
      if (full != nullptr && n < rows) full[(cpos * rows + n) * (int64_t)(C * R3) + ff] = pb;
    }
  }
  best = umax64(best, shfl_xor64(best, 32));
  if (lane < 32 && n < rows) atomicMax(&packed[cpos * rows + n], best);
}


__global__ void k_fill_u64(unsigned long long *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

__global__ void k_unpack(const unsigned long long *__restrict__ packed, int64_t n,
                         float *__restrict__ pmax, int32_t *__restrict__ argf) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned long long v = packed[i];
  pmax[i] = __uint_as_float((unsigned)(v >> 32));
  argf[i] = (int32_t)(0xffffffffu - (unsigned)v);
}

template <class Op, int SPLIT>
hipError_t launch_t(dsgrft_plan p, const void *F, int fsc, int64_t nunits,
                    int64_t unit0, float *full, hipStream_t s) {
  using CF = Cfg<Op, SPLIT>;
  int64_t tiles = nunits * (p->NB / CF::NBG) * (p->FB / 4);
  const int32_t *gsc = Op::FR == 2 ? p->g_scale : nullptr;
  const int32_t *gsh = std::is_same<Op, OpF16>::value ? p->g_shift : nullptr;
  hipLaunchKernelGGL((k_fine_mfma<Op, SPLIT>), dim3((unsigned)tiles), dim3(256), 0, s,
                     (const uint4 *)F, (const uint4 *)p->G, gsc, fsc, gsh, p->packed, full,
                     p->FB, p->NB, p->Mp / Op::KSTEP, p->rows_p, nunits, unit0, p->R3,
                     p->C, p->rows, 8);
  return hipGetLastError();
}

template <class Op>
hipError_t launch_split(dsgrft_plan p, const void *F, int fsc, int split,
                        int64_t nunits, int64_t unit0, float *full, hipStream_t s) {
  switch (split) {
    case 1: return launch_t<Op, 1>(p, F, fsc, nunits, unit0, full, s);
    case 2: return launch_t<Op, 2>(p, F, fsc, nunits, unit0, full, s);
    case 3: return launch_t<Op, 3>(p, F, fsc, nunits, unit0, full, s);
    case 4: return launch_t<Op, 4>(p, F, fsc, nunits, unit0, full, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_fill_u64(unsigned long long *ptr, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     ptr, n);
  return hipGetLastError();
}

hipError_t launch_unpack(dsgrft_plan p, int64_t ncells, float *pmax,
                         int32_t *argf, hipStream_t s) {
  int64_t n = ncells * p->rows;
  hipLaunchKernelGGL(k_unpack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     p->packed, n, pmax, argf);
  return hipGetLastError();
}

hipError_t launch_fine_mfma(dsgrft_plan p, dsgrft_form form, int split,
                            int64_t nunits, int64_t unit0, float *full,
                            hipStream_t s) {
  switch (form) {
    case DSGRFT_FORM_F16:
      return launch_split<OpF16>(p, p->F16, 0, split, nunits, unit0, full, s);
    case DSGRFT_FORM_F16_3M: {
      // K steps go in pairs: Mp is a multiple of 64, so Mp / 16 is even
      if (split != 1 || (p->Mp / OpF16::KSTEP) % 2 != 0) return hipErrorInvalidValue;
      const int64_t tiles = nunits * (p->NB / 4) * (p->FB / 4);
      hipLaunchKernelGGL(k_fine_mfma3, dim3((unsigned)tiles), dim3(256), 0, s,
                         (const uint4 *)p->F16, (const uint4 *)p->G, p->g_shift, p->packed,
                         full, p->FB,
                         p->NB, p->Mp / OpF16::KSTEP, nunits, unit0, p->R3, p->C, p->rows, 8);
      return hipGetLastError();
    }
    case DSGRFT_FORM_F16_SYM:
    case DSGRFT_FORM_BF16_SYM: {
      const bool b = form == DSGRFT_FORM_BF16_SYM;
      if ((b ? (split != 2 && split != 3) : split != 1) || (p->Mp / OpF16::KSTEP) % 2 != 0 ||
          p->FBs <= 0 || p->FBs % 2 != 0 || p->NB % 4 != 0)
        return hipErrorInvalidValue;
      const int64_t tiles = nunits * (p->NB / 4) * (p->FBs / 2);
#define DS_SYM(OP, NPF, NPG, TAB, SH)                                                   \
  hipLaunchKernelGGL((k_fine_mfma_sym<OP, NPF, NPG>), dim3((unsigned)tiles), dim3(256), 0, s, \
                     (const uint4 *)(TAB), (const uint4 *)p->G, p->sym_cols, SH, p->packed,  \
                     full, p->FBs, p->NB, p->Mp / OP::KSTEP, nunits, unit0, p->R3, p->C,     \
                     p->rows, 4)
      if (!b)
        DS_SYM(OpF16, 2, 2, p->FS16, p->g_shift);
      else if (split == 2)
        DS_SYM(OpBF16, 2, 4, p->FSB16, nullptr);
      else
        DS_SYM(OpBF16, 4, 4, p->FSB16, nullptr);
#undef DS_SYM
      return hipGetLastError();
    }
    case DSGRFT_FORM_BF16:
      return launch_split<OpBF16>(p, p->FBF16, 0, split, nunits, unit0, full, s);
    case DSGRFT_FORM_BF16_GLO:
      if (split != 2) return hipErrorInvalidValue;
      return launch_t<OpBF16, SPLIT_GLO>(p, p->FBF16, 0, nunits, unit0, full, s);
    case DSGRFT_FORM_FP8:
      // fine table: hi = e4m3(256 F) -> 2^-8 (code 119), lo -> 2^-12
      return launch_split<OpF8>(p, p->F8, 119, split, nunits, unit0, full, s);
    case DSGRFT_FORM_FP8_SYM: {
      if ((split != 3 && split != 4) || p->FS8 == nullptr || p->FBs <= 0 || p->FBs % 2 != 0 ||
          p->NB % 4 != 0)
        return hipErrorInvalidValue;
      const int64_t tiles = nunits * (p->NB / 4) * (p->FBs / 2);
#define DS_SYM8(SP)                                                                        \
  hipLaunchKernelGGL((k_fine_mfma_sym8<SP>), dim3((unsigned)tiles), dim3(512), 0, s,         \
                     (const uint4 *)p->FS8, (const uint4 *)p->G, p->g_scale, 119,           \
                     p->sym_cols, p->packed, full, p->FBs, p->NB, p->Mp / OpF8::KSTEP,      \
                     p->rows_p, nunits, unit0, p->R3, p->C, p->rows, 4)
      if (split == 3)
        DS_SYM8(3);
      else
        DS_SYM8(4);
#undef DS_SYM8
      return hipGetLastError();
    }
    default:
      return hipErrorInvalidValue;
  }
}
