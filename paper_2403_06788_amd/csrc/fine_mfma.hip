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
// and with the hi+lo split of both operands (split = 3) the three products
// hi*hi + hi*lo + lo*hi of each, all accumulated in FP32.
//
// Work decomposition: a workgroup of 2 x 2 waves computes a 128 (fine) x
// 64 WNB (row) tile of one unit; each wave a 64 x 32 WNB sub-tile as 2 x WNB
// blocks of v_mfma_f32_32x32x16 (fine cells on the MFMA rows, range rows on
// its columns), WNB = 4 for one product per operand pair and 2 for the
// three-product split.  The wider wave tile reuses each fragment read from
// LDS for more MFMAs: the kernel is bound by LDS traffic (copies in plus
// fragment reads), not by the MFMA issue.  Accumulators live in AGPRs.
// Operand fragments are stored pre-swizzled in global memory.
//
// Pipeline (one K step = 16 pulses):
//  * operands move global -> LDS with direct LDS-DMA loads (16 bytes per
//    lane; one 1 KiB fragment per wave and chunk row), into a ring of NST
//    stages issued NST - 1 steps ahead;
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
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void;
typedef const __attribute__((address_space(1))) void glob_void;

template <typename T>
struct Mfma;
template <>
struct Mfma<_Float16> {
  static __device__ inline f16v run(uint4 a, uint4 b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(h8, a),
                                                  __builtin_bit_cast(h8, b), c, 0, 0, 0);
  }
};
template <>
struct Mfma<__bf16> {
  static __device__ inline f16v run(uint4 a, uint4 b, f16v c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(b8, a),
                                                   __builtin_bit_cast(b8, b), c, 0, 0, 0);
  }
};

__device__ inline uint4 neg16(uint4 a) {
  return make_uint4(a.x ^ 0x80008000u, a.y ^ 0x80008000u, a.z ^ 0x80008000u,
                    a.w ^ 0x80008000u);
}

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

template <int SPLIT>
struct Cfg {
  static constexpr int NP = SPLIT == 1 ? 2 : 4;   // operand planes
  static constexpr int WNB = 2;                   // row blocks per wave
  static constexpr int NBLK = 4 + 2 * WNB;        // fragments per plane/stage
  static constexpr int NST = SPLIT == 1 ? 4 : 3;  // LDS ring stages
  static constexpr int MINB = SPLIT == 1 ? 2 : 1; // workgroups per CU
  static constexpr int CH = NP * NBLK * 64;       // 16-byte chunks per stage
  static constexpr int CPT = CH / 256;            // chunks per thread
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
template <int NP, int WNB, int SPLIT>
__device__ inline void order_step() {
  __builtin_amdgcn_sched_group_barrier(0x100, NP * (2 + WNB), 0);  // DS reads
  __builtin_amdgcn_sched_group_barrier(0x008, SPLIT * 8 * WNB, 0); // MFMAs
}

template <int NP, int WNB>
__device__ inline void read_frags(const uint4 *__restrict__ slot, int wf, int wn,
                                  int lane, uint4 (&a)[NP][2], uint4 (&b)[NP][WNB]) {
  constexpr int NBLK = 4 + 2 * WNB;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
#pragma unroll
    for (int i = 0; i < 2; ++i) a[p][i] = slot[(p * NBLK + wf * 2 + i) * 64 + lane];
#pragma unroll
    for (int j = 0; j < WNB; ++j)
      b[p][j] = slot[(p * NBLK + 4 + wn * WNB + j) * 64 + lane];
  }
}

// Empty asm "redefining" a fragment set: MFMAs that consume the set cannot
// be scheduled above this point.  Placed after each step's barrier, it keeps
// the next step's MFMAs (and the waits for their LDS reads) out of the
// current step.
template <int NP, int WNB>
__device__ inline void pin(uint4 (&a)[NP][2], uint4 (&b)[NP][WNB]) {
#pragma unroll
  for (int p = 0; p < NP; ++p) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
      asm volatile("" : "+v"(a[p][i].x), "+v"(a[p][i].y), "+v"(a[p][i].z), "+v"(a[p][i].w));
#pragma unroll
    for (int j = 0; j < WNB; ++j)
      asm volatile("" : "+v"(b[p][j].x), "+v"(b[p][j].y), "+v"(b[p][j].z), "+v"(b[p][j].w));
  }
}

template <typename T, int SPLIT, int NP, int WNB>
__device__ inline void mma_step(const uint4 (&a)[NP][2], const uint4 (&b)[NP][WNB],
                                f16v (&accR)[2][WNB], f16v (&accI)[2][WNB]) {
#pragma unroll
  for (int s = 0; s < SPLIT; ++s) {
    const int pa = (s == 2) ? 2 : 0;  // hi*hi, hi*lo, lo*hi
    const int pb = (s == 1) ? 2 : 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const uint4 nfi = neg16(a[pa + 1][i]);
#pragma unroll
      for (int j = 0; j < WNB; ++j) {
        accR[i][j] = Mfma<T>::run(a[pa][i], b[pb][j], accR[i][j]);
        accR[i][j] = Mfma<T>::run(nfi, b[pb + 1][j], accR[i][j]);
        accI[i][j] = Mfma<T>::run(a[pa][i], b[pb + 1][j], accI[i][j]);
        accI[i][j] = Mfma<T>::run(a[pa + 1][i], b[pb][j], accI[i][j]);
      }
    }
  }
}

template <typename T, int SPLIT>
__global__ __launch_bounds__(256, Cfg<SPLIT>::MINB) void k_fine_mfma(
    const uint4 *__restrict__ F, const uint4 *__restrict__ G,
    unsigned long long *__restrict__ packed, float *__restrict__ full, int FB,
    int NB, int KB, int64_t nunits, int64_t unit0, int R3, int C, int rows,
    int GN) {
  using CF = Cfg<SPLIT>;
  constexpr int NP = CF::NP, NST = CF::NST, CH = CF::CH, CPT = CF::CPT;
  constexpr int WNB = CF::WNB, NBLK = CF::NBLK;
  __shared__ uint4 lds[NST][CH];

  const int NT = NB / (2 * WNB), FT = FB >> 2;
  const TileMap tm = map_tile(blockIdx.x, nunits * NT * FT, NT, FT, GN);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wf = wave & 1, wn = wave >> 1;
  const int wbase = tid & ~63;

  // Global source of this thread's chunks (16-byte units).  Chunk c of a
  // stage: lane c % 64, block (c / 64) % NBLK (0-3 fine, then rows), plane
  // (c / 64) / NBLK.
  const uint4 *src[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int c = tid + 256 * j;
    const int ln = c & 63, blk = (c >> 6) % NBLK, plane = (c >> 6) / NBLK;
    src[j] = (blk < 4)
                 ? F + (((int64_t)plane * FB + tm.ft * 4 + blk) * KB) * 64 + ln
                 : G + (((tm.u * NP + plane) * NB + tm.nt * 2 * WNB + (blk - 4)) * (int64_t)KB) * 64 + ln;
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

  f16v accR[2][WNB], accI[2][WNB];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < WNB; ++j) {
      accR[i][j] = f16v{};
      accI[i][j] = f16v{};
    }

  const int nkt = KB;
  // prologue: stages 0 .. NST-2 in flight, stage 0 visible, its fragments read
#pragma unroll
  for (int s = 0; s < NST - 1; ++s)
    if (s < nkt) issue(s);
  wait_copies_barrier<CPT>((nkt - 1 < NST - 2) ? nkt - 1 : NST - 2);
  uint4 a0[NP][2], b0[NP][WNB], a1[NP][2], b1[NP][WNB];
  read_frags<NP, WNB>(lds[0], wf, wn, lane, a0, b0);

  // One K step: make stage kt+1 visible, read its fragments into (an, bn),
  // refill the slot freed one step ago, then the MFMAs of step kt.
#define DS_STEP(KT, AC, BC, AN, BN)                                              \
  do {                                                                         \
    const int kt_ = (KT);                                                      \
    if (kt_ + 1 < nkt) {                                                       \
      const int last = (nkt - 1 < kt_ + NST - 2) ? nkt - 1 : kt_ + NST - 2;    \
      wait_copies_barrier<CPT>(last - (kt_ + 1));                              \
      pin<NP, WNB>(AC, BC);                                                    \
      read_frags<NP, WNB>(lds[(kt_ + 1) % NST], wf, wn, lane, AN, BN);         \
      if (kt_ + NST - 1 < nkt) issue(kt_ + NST - 1);                           \
    }                                                                          \
    mma_step<T, SPLIT, NP, WNB>(AC, BC, accR, accI);                           \
  } while (0)

  // Steady state, branch-free: every step waits for the same number of
  // copies in flight and refills a slot.
#define DS_STEADY(KT, AC, BC, AN, BN)                                          \
  do {                                                                         \
    const int kt_ = (KT);                                                      \
    wait_copies_barrier<CPT>(NST - 3);                                         \
    pin<NP, WNB>(AC, BC);                                                      \
    read_frags<NP, WNB>(lds[(kt_ + 1) % NST], wf, wn, lane, AN, BN);           \
    issue(kt_ + NST - 1);                                                      \
    mma_step<T, SPLIT, NP, WNB>(AC, BC, accR, accI);                           \
    order_step<NP, WNB, SPLIT>();                                              \
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
  const int64_t ug = unit0 + tm.u;
  const int64_t cpos = ug / R3;
  const unsigned fbase = (unsigned)((ug % R3) * C);
#pragma unroll
  for (int j = 0; j < WNB; ++j) {
    const int n = (tm.nt * 2 * WNB + wn * WNB + j) * 32 + (lane & 31);
    unsigned long long best = 0ull;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int fb0 = (tm.ft * 4 + wf * 2 + i) * 32 + 4 * (lane >> 5);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = fb0 + 8 * (r >> 2) + (r & 3);
        const float yr = accR[i][j][r], yi = accI[i][j][r];
        const float pw = yr * yr + yi * yi;
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

template <typename T, int SPLIT>
hipError_t launch_t(dsgrft_plan p, int64_t nunits, int64_t unit0, float *full,
                    hipStream_t s) {
  int64_t tiles = nunits * (p->NB / (2 * Cfg<SPLIT>::WNB)) * (p->FB / 4);
  hipLaunchKernelGGL((k_fine_mfma<T, SPLIT>), dim3((unsigned)tiles), dim3(256), 0, s,
                     (const uint4 *)(std::is_same<T, _Float16>::value ? p->F16 : p->FBF16),
                     (const uint4 *)p->G, p->packed, full, p->FB, p->NB, p->KB,
                     nunits, unit0, p->R3, p->C, p->rows, 8);
  return hipGetLastError();
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
  if (form == DSGRFT_FORM_F16)
    return split == 1 ? launch_t<_Float16, 1>(p, nunits, unit0, full, s)
                      : launch_t<_Float16, 3>(p, nunits, unit0, full, s);
  if (form == DSGRFT_FORM_BF16)
    return split == 1 ? launch_t<__bf16, 1>(p, nunits, unit0, full, s)
                      : launch_t<__bf16, 3>(p, nunits, unit0, full, s);
  return hipErrorInvalidValue;
}
