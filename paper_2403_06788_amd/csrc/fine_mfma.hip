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
// Work decomposition: a workgroup of 4 waves computes a 128 (fine) x 128
// (row) tile of one unit; each wave a 64 x 64 sub-tile as 2 x 2 blocks of
// v_mfma_f32_32x32x16 (fine cells on the MFMA rows, range rows on its
// columns).  Operand fragments are stored pre-swizzled in global memory, are
// staged through LDS with one 16-byte load and store per lane and fragment
// (double-buffered, one barrier per K step) and are read back lane-linearly.
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

template <typename T, int SPLIT>
__global__ __launch_bounds__(256, 2) void k_fine_mfma(
    const uint4 *__restrict__ F, const uint4 *__restrict__ G,
    unsigned long long *__restrict__ packed, float *__restrict__ full, int FB,
    int NB, int KB, int64_t nunits, int64_t unit0, int R3, int C, int rows,
    int GN) {
  constexpr int NP = SPLIT == 1 ? 2 : 4;      // operand planes
  constexpr int KBT = SPLIT == 1 ? 2 : 1;     // 16-pulse blocks per K step
  constexpr int CH = NP * 8 * KBT * 64;       // 16-byte chunks per stage
  constexpr int CPT = CH / 256;               // chunks per thread
  __shared__ uint4 lds[2][CH];

  const int NT = NB >> 2, FT = FB >> 2;
  const TileMap tm = map_tile(blockIdx.x, nunits * NT * FT, NT, FT, GN);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wf = wave & 1, wn = wave >> 1;

  // global source offsets of this thread's chunks (in 16-byte units)
  int64_t src[CPT];
  bool isF[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int c = tid + 256 * j;
    const int ln = c & 63;
    int rest = c >> 6;
    const int kbt = rest % KBT;
    rest /= KBT;
    const int blk = rest & 7, plane = rest >> 3;
    isF[j] = blk < 4;
    if (blk < 4)
      src[j] = (((int64_t)plane * FB + tm.ft * 4 + blk) * KB + kbt) * 64 + ln;
    else
      src[j] = (((tm.u * NP + plane) * NB + tm.nt * 4 + (blk - 4)) * (int64_t)KB + kbt) * 64 + ln;
  }

  f16v accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = f16v{};
      accI[i][j] = f16v{};
    }

  const int nkt = KB / KBT;
  {
    uint4 st[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) st[j] = isF[j] ? F[src[j]] : G[src[j]];
#pragma unroll
    for (int j = 0; j < CPT; ++j) lds[0][tid + 256 * j] = st[j];
  }
  __syncthreads();

  for (int kt = 0; kt < nkt; ++kt) {
    const int cur = kt & 1;
    // prefetch the next K step (the last iteration re-reads its own step;
    // the copy it stores into the idle buffer is never read)
    const int64_t step = (int64_t)((kt + 1 < nkt) ? kt + 1 : kt) * KBT * 64;
    uint4 st[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) st[j] = isF[j] ? F[src[j] + step] : G[src[j] + step];
#pragma unroll
    for (int kbt = 0; kbt < KBT; ++kbt) {
      uint4 a[NP][2], b[NP][2];
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a[p][i] = lds[cur][((p * 8 + wf * 2 + i) * KBT + kbt) * 64 + lane];
          b[p][i] = lds[cur][((p * 8 + 4 + wn * 2 + i) * KBT + kbt) * 64 + lane];
        }
#pragma unroll
      for (int s = 0; s < SPLIT; ++s) {
        const int pa = (s == 2) ? 2 : 0;   // hi*hi, hi*lo, lo*hi
        const int pb = (s == 1) ? 2 : 0;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const uint4 nfi = neg16(a[pa + 1][i]);
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            accR[i][j] = Mfma<T>::run(a[pa][i], b[pb][j], accR[i][j]);
            accR[i][j] = Mfma<T>::run(nfi, b[pb + 1][j], accR[i][j]);
            accI[i][j] = Mfma<T>::run(a[pa][i], b[pb + 1][j], accI[i][j]);
            accI[i][j] = Mfma<T>::run(a[pa + 1][i], b[pb][j], accI[i][j]);
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) lds[cur ^ 1][tid + 256 * j] = st[j];
    __syncthreads();
  }

  // ---- epilogue: |Y|^2, best fine cell per row, merge -----------------
  const int64_t ug = unit0 + tm.u;
  const int64_t cpos = ug / R3;
  const unsigned fbase = (unsigned)((ug % R3) * C);
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int n = (tm.nt * 4 + wn * 2 + j) * 32 + (lane & 31);
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
  int64_t tiles = nunits * (p->NB / 4) * (p->FB / 4);
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
