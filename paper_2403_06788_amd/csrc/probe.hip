// Attainable matrix-core rate, for the roofline of the fine search (a
// measurement aid, not part of the method).
//
// The published dense peak assumes the nominal clock.  Under sustained
// matrix work on random data the chip runs at a power-limited clock, so the
// rate a kernel can reach depends on its operands.  This probe measures it:
// every wave keeps random A and B fragments (eight each for fp16 and bf16,
// four each of twice the size for e4m3) and eight accumulators in registers
// and issues v_mfma_f32_32x32x16_{f16,bf16} or
// v_mfma_scale_f32_32x32x64_f8f6f4 back to back, each MFMA taking another
// operand pair (the B fragment rotates against the A fragment), with no
// memory traffic.  Operands are finite values with random signs, mantissas
// and exponents in [2^-8, 2^1) for fp16 and bf16, the magnitudes of the
// search's phasors and scaled gathered rows, and in [2^-1, 2^8) for e4m3
// (the 8-bit form's scaled operands, no NaN code), with the E8M0 block
// scales of that form (2^-8 for A, 2^-7 for B).  Thread 0 of
// every workgroup reads the shader clock counter and the constant 100 MHz
// real-time counter at its start and end, giving the mean clock while the
// loop runs.
#include <vector>

#include "internal.h"

namespace {

typedef _Float16 ph8 __attribute__((ext_vector_type(8)));
typedef __bf16 pb8 __attribute__((ext_vector_type(8)));
typedef float pf16v __attribute__((ext_vector_type(16)));
typedef int pi8v __attribute__((ext_vector_type(8)));

enum { P_F16 = 0, P_BF16 = 1, P_FP8 = 2 };

__device__ inline unsigned xs32(unsigned &s) {
  s ^= s << 13;
  s ^= s >> 17;
  s ^= s << 5;
  return s;
}

// Two random 16-bit floats in one word: sign, exponent field in
// [E0, E0 + 8], mantissa (M bits).
template <int E0, int MB>
__device__ inline unsigned rand_pair(unsigned &s) {
  unsigned w = 0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const unsigned r = xs32(s);
    const unsigned e = E0 + (r >> 4) % 9u;
    const unsigned v = ((r & 1u) << 15) | (e << MB) | ((r >> 8) & ((1u << MB) - 1u));
    w |= v << (16 * h);
  }
  return w;
}

// Four random e4m3 values in one word: sign, exponent field in [6, 14]
// (2^-1 .. 2^7 before the block scale; 15 would allow the NaN code), three
// mantissa bits.
__device__ inline unsigned rand_quad_e4m3(unsigned &s) {
  unsigned w = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const unsigned r = xs32(s);
    const unsigned e = 6u + (r >> 4) % 9u;
    w |= (((r & 1u) << 7) | (e << 3) | ((r >> 8) & 7u)) << (8 * q);
  }
  return w;
}

// One operand fragment per lane: 16 bytes (fp16, bf16) or 32 bytes (e4m3).
template <int T>
struct PFrag {
  uint4 v[T == P_FP8 ? 2 : 1];
};

template <int T>
__device__ inline PFrag<T> rand_frag(unsigned &s) {
  PFrag<T> f;
#pragma unroll
  for (int h = 0; h < (T == P_FP8 ? 2 : 1); ++h) {
    if constexpr (T == P_FP8)
      f.v[h] = make_uint4(rand_quad_e4m3(s), rand_quad_e4m3(s), rand_quad_e4m3(s),
                          rand_quad_e4m3(s));
    else if constexpr (T == P_BF16)  // exponent field 119..127, 7 mantissa bits
      f.v[h] = make_uint4(rand_pair<119, 7>(s), rand_pair<119, 7>(s), rand_pair<119, 7>(s),
                          rand_pair<119, 7>(s));
    else  // fp16: exponent field 7..15 (2^-8 .. 2^0), 10 mantissa bits
      f.v[h] = make_uint4(rand_pair<7, 10>(s), rand_pair<7, 10>(s), rand_pair<7, 10>(s),
                          rand_pair<7, 10>(s));
  }
  return f;
}

template <int T>
__device__ inline pf16v mma(const PFrag<T> &a, const PFrag<T> &b, pf16v c) {
  if constexpr (T == P_FP8) {
    const pi8v A = {(int)a.v[0].x, (int)a.v[0].y, (int)a.v[0].z, (int)a.v[0].w,
                    (int)a.v[1].x, (int)a.v[1].y, (int)a.v[1].z, (int)a.v[1].w};
    const pi8v B = {(int)b.v[0].x, (int)b.v[0].y, (int)b.v[0].z, (int)b.v[0].w,
                    (int)b.v[1].x, (int)b.v[1].y, (int)b.v[1].z, (int)b.v[1].w};
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, B, c, 0, 0, 0, 119, 0, 120);
  } else if constexpr (T == P_BF16) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(pb8, a.v[0]),
                                                   __builtin_bit_cast(pb8, b.v[0]), c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(ph8, a.v[0]),
                                                  __builtin_bit_cast(ph8, b.v[0]), c, 0, 0, 0);
  }
}

template <int T>
__global__ __launch_bounds__(256) void k_mfma_probe(int iters, unsigned seed,
                                                    float *__restrict__ sink,
                                                    unsigned long long *__restrict__ clk) {
  constexpr int NF = T == P_FP8 ? 4 : 8;  // A and B fragments per wave
  unsigned s = seed ^ (blockIdx.x * 2654435761u) ^ (threadIdx.x * 40503u);
  if (s == 0) s = 1;
  PFrag<T> a[NF], b[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    a[i] = rand_frag<T>(s);
    b[i] = rand_frag<T>(s);
  }
  pf16v acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = pf16v{};
  unsigned long long t0 = 0, r0 = 0;
  if (threadIdx.x == 0) {
    t0 = __builtin_amdgcn_s_memtime();
    r0 = __builtin_amdgcn_s_memrealtime();
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int i = 0; i < 8; ++i) acc[i] = mma<T>(a[i % NF], b[(i + r) % NF], acc[i]);
  }
  if (threadIdx.x == 0) {
    const unsigned long long t1 = __builtin_amdgcn_s_memtime();
    const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
    clk[2 * blockIdx.x] = t1 - t0;
    clk[2 * blockIdx.x + 1] = r1 - r0;
  }
  float sum = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) sum += acc[i][e];
  sink[(int64_t)blockIdx.x * 256 + threadIdx.x] = sum;
}

constexpr int kProbeBlocks = 2048;

}  // namespace

extern "C" dsgrft_status dsgrft_mfma_probe(dsgrft_form form, double ms, double *h_tflops,
                                           double *h_ghz) {
  if (!h_tflops || !h_ghz || !(ms >= 1.0 && ms <= 10000.0)) return DSGRFT_E_INVALID;
  if (form != DSGRFT_FORM_F16 && form != DSGRFT_FORM_BF16 && form != DSGRFT_FORM_FP8)
    return DSGRFT_E_INVALID;
  float *sink = nullptr;
  unsigned long long *clk = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  dsgrft_status st = DSGRFT_E_DEVICE;
  std::vector<unsigned long long> h(2 * kProbeBlocks);
  auto launch = [&](int iters) {
    if (form == DSGRFT_FORM_FP8)
      hipLaunchKernelGGL(k_mfma_probe<P_FP8>, dim3(kProbeBlocks), dim3(256), 0, nullptr, iters,
                         12345u, sink, clk);
    else if (form == DSGRFT_FORM_BF16)
      hipLaunchKernelGGL(k_mfma_probe<P_BF16>, dim3(kProbeBlocks), dim3(256), 0, nullptr, iters,
                         12345u, sink, clk);
    else
      hipLaunchKernelGGL(k_mfma_probe<P_F16>, dim3(kProbeBlocks), dim3(256), 0, nullptr, iters,
                         12345u, sink, clk);
    return hipGetLastError();
  };
  // 64 MFMAs per wave and iteration, 4 waves per workgroup; K = 16 (fp16,
  // bf16) or 64 (e4m3) per MFMA
  const double kdim = form == DSGRFT_FORM_FP8 ? 64.0 : 16.0;
  const double flops_per_iter = (double)kProbeBlocks * 4 * 64 * 32.0 * 32.0 * kdim * 2.0;
  float t_ms = 0.f;
  int iters = 64;
  if (hipMalloc((void **)&sink, (size_t)kProbeBlocks * 256 * sizeof(float)) != hipSuccess ||
      hipMalloc((void **)&clk, h.size() * sizeof(unsigned long long)) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    goto done;
  // warm-up, then size the timed run to about `ms` milliseconds
  if (launch(iters) != hipSuccess || hipEventRecord(e0, nullptr) != hipSuccess ||
      launch(iters) != hipSuccess || hipEventRecord(e1, nullptr) != hipSuccess ||
      hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t_ms, e0, e1) != hipSuccess)
    goto done;
  iters = (int)(iters * ms / (t_ms > 0.01f ? t_ms : 0.01f));
  iters = iters < 64 ? 64 : (iters > (1 << 22) ? (1 << 22) : iters);
  if (hipEventRecord(e0, nullptr) != hipSuccess || launch(iters) != hipSuccess ||
      hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(&t_ms, e0, e1) != hipSuccess ||
      hipMemcpy(h.data(), clk, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost) !=
          hipSuccess)
    goto done;
  {
    double cyc = 0.0, real = 0.0;
    for (int b = 0; b < kProbeBlocks; ++b) {
      cyc += (double)h[2 * b];
      real += (double)h[2 * b + 1];
    }
    *h_tflops = flops_per_iter * iters / (t_ms * 1e-3) / 1e12;
    *h_ghz = real > 0.0 ? cyc / real * 0.1 : 0.0;  // real-time counter: 100 MHz
    st = DSGRFT_OK;
  }
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (sink) (void)hipFree(sink);
  if (clk) (void)hipFree(clk);
  (void)hipGetLastError();
  return st;
}
