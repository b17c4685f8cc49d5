// Instruction rates and reciprocal accuracy on gfx950: the figures behind
// the issue-slot model of the evaluation kernels.
//
//   throughput  every lane runs 8 independent chains of one operation for
//               `iters` iterations; the grid holds 32 waves per CU, so
//               dependent latency is hidden and the rate is the issue rate.
//               Reported as wave64 instructions per cycle per CU at the
//               published 2.4 GHz clock (after a warm-up that lets the clock
//               ramp up), and relative to v_fma_f64.
//   accuracy    v_rcp_f64 and v_rcp_f32 against the correctly rounded
//               1/x of the same format, over values with random mantissas
//               across 2^-60 .. 2^60: the largest relative error.
//
// Build and run: python -m paper_1606_06508_amd.isa_rates
// Every kernel writes one value per thread inside its output array.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CK(x)                                                                        \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) {                                                          \
      std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
      std::exit(1);                                                                  \
    }                                                                                \
  } while (0)

constexpr int kChains = 8;

enum Op {
  FMA64,
  MUL64,
  ADD64,
  RCP64,
  DIV64,
  FMA32,
  RCP32,
  DIV32,
  kOps
};
static const char* kNames[kOps] = {"v_fma_f64",  "v_mul_f64", "v_add_f64",
                                   "v_rcp_f64",  "f64 IEEE divide (1/x)",
                                   "v_fmac_f32 (VOP2, VGPR operands)",
                                   "v_rcp_f32", "f32 IEEE divide (1/x)"};

// Chains start near 1 and stay finite for any iteration count: the binary64
// multiply-adds contract towards a fixed point, the binary32 ones grow
// linearly, reciprocals alternate, and the multiply and add chains undo
// each step.
template <int OP>
__global__ void __launch_bounds__(256) k_rate(double* out, int iters, double seed) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const double lane = 1e-3 * (double)(threadIdx.x & 63);  // per-lane operands (VGPRs)
  if constexpr (OP >= FMA32) {
    float a[kChains];
    const float b = 0.5f + (float)lane, c = 0.25f + (float)lane;
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = (float)seed + 0.01f * i;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < kChains; ++i) {
        // accumulator form a += b c, as in the kernels' sums: VOP2 v_fmac_f32
        if constexpr (OP == FMA32) a[i] = __builtin_fmaf(b, c, a[i]);
        if constexpr (OP == RCP32) a[i] = __builtin_amdgcn_rcpf(a[i]);
        if constexpr (OP == DIV32) a[i] = 1.0f / a[i];
      }
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += a[i];
    out[tid] = s;
  } else {
    double a[kChains];
    const double b = 0.5 + lane, c = 0.25 + lane;
    const double q = 1.0 + lane, qi = 1.0 / q;
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = seed + 0.01 * i;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < kChains; ++i) {
        if constexpr (OP == FMA64) a[i] = __builtin_fma(a[i], b, c);
        if constexpr (OP == MUL64) a[i] = (a[i] * q) * qi;  // two multiplies, bounded
        if constexpr (OP == ADD64) a[i] = (a[i] + c) - c;   // two adds, bounded
        if constexpr (OP == RCP64) a[i] = __builtin_amdgcn_rcp(a[i]);
        if constexpr (OP == DIV64) a[i] = 1.0 / a[i];
      }
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kChains; ++i) s += a[i];
    out[tid] = s;
  }
}

__global__ void __launch_bounds__(256)
    k_rcp_accuracy(const double* __restrict__ v, int n, double* __restrict__ e64,
                   double* __restrict__ e32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = v[i];
  const double r = __builtin_amdgcn_rcp(x), q = 1.0 / x;
  e64[i] = fabs(r - q) / fabs(q);
  const float xf = (float)x;
  const float rf = __builtin_amdgcn_rcpf(xf), qf = 1.0f / xf;
  e32[i] = fabs((double)rf - (double)qf) / fabs((double)qf);
}

template <int OP>
static double time_op(double* out, int blocks, int iters) {
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  k_rate<OP><<<blocks, 256>>>(out, iters, 1.0);  // warm-up
  CK(hipGetLastError());
  CK(hipEventRecord(e0));
  k_rate<OP><<<blocks, 256>>>(out, iters, 1.0);
  CK(hipEventRecord(e1));
  CK(hipEventSynchronize(e1));
  float ms = 0.0f;
  CK(hipEventElapsedTime(&ms, e0, e1));
  CK(hipEventDestroy(e0));
  CK(hipEventDestroy(e1));
  return ms;
}

int main() {
  int dev = 0, cus = 0;
  CK(hipSetDevice(dev));
  CK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = cus * 8;  // 8 blocks of 4 waves: 32 waves per CU
  const int iters = 32768;
  double* out = nullptr;
  CK(hipMalloc(&out, sizeof(double) * blocks * 256));
  // the clock needs tens of milliseconds of steady work to ramp up
  for (int w = 0; w < 40; ++w) k_rate<FMA64><<<blocks, 256>>>(out, iters, 1.0);
  CK(hipGetLastError());
  CK(hipDeviceSynchronize());
  const double waves = blocks * 4.0;
  const double instr = waves * (double)iters * kChains;  // wave instructions of the op
  const double clock = 2.4e9;
  double ms[kOps];
  ms[FMA64] = time_op<FMA64>(out, blocks, iters);
  ms[MUL64] = time_op<MUL64>(out, blocks, iters);
  ms[ADD64] = time_op<ADD64>(out, blocks, iters);
  ms[RCP64] = time_op<RCP64>(out, blocks, iters);
  ms[DIV64] = time_op<DIV64>(out, blocks, iters);
  ms[FMA32] = time_op<FMA32>(out, blocks, iters);
  ms[RCP32] = time_op<RCP32>(out, blocks, iters);
  ms[DIV32] = time_op<DIV32>(out, blocks, iters);
  std::printf("CUs %d, 32 waves per CU, %d iterations x %d chains per lane\n", cus, iters, kChains);
  std::printf("%-36s %12s %18s %14s\n", "operation", "ms", "wave instr/cyc/CU", "vs v_fma_f64");
  for (int o = 0; o < kOps; ++o) {
    const double per = (o == MUL64 || o == ADD64) ? 2.0 : 1.0;  // operations per chain step
    const double rate = per * instr / (ms[o] * 1e-3) / clock / cus;
    std::printf("%-36s %12.3f %18.3f %14.3f\n", kNames[o], ms[o], rate,
                per * ms[FMA64] / ms[o]);
  }

  // reciprocal accuracy
  const int n = 1 << 20;
  std::vector<double> v(n);
  uint64_t s = 0x9E3779B97F4A7C15ull;
  for (int i = 0; i < n; ++i) {
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    const double mant = 1.0 + (double)(s >> 11) * 0x1p-53;  // [1, 2)
    const int ex = (int)((s >> 3) % 121) - 60;               // 2^-60 .. 2^60
    v[i] = std::ldexp(mant, ex) * ((s & 1) ? -1.0 : 1.0);
  }
  double *dv, *e64, *e32;
  CK(hipMalloc(&dv, sizeof(double) * n));
  CK(hipMalloc(&e64, sizeof(double) * n));
  CK(hipMalloc(&e32, sizeof(double) * n));
  CK(hipMemcpy(dv, v.data(), sizeof(double) * n, hipMemcpyHostToDevice));
  k_rcp_accuracy<<<(n + 255) / 256, 256>>>(dv, n, e64, e32);
  CK(hipGetLastError());
  std::vector<double> h64(n), h32(n);
  CK(hipMemcpy(h64.data(), e64, sizeof(double) * n, hipMemcpyDeviceToHost));
  CK(hipMemcpy(h32.data(), e32, sizeof(double) * n, hipMemcpyDeviceToHost));
  double m64 = 0.0, m32 = 0.0;
  for (int i = 0; i < n; ++i) {
    m64 = std::fmax(m64, h64[i]);
    m32 = std::fmax(m32, h32[i]);
  }
  std::printf("v_rcp_f64 max relative error %.3e = 2^%.2f (vs correctly rounded 1/x, %d values)\n",
              m64, std::log2(m64), n);
  std::printf("v_rcp_f32 max relative error %.3e = 2^%.2f (u32 = 2^-24)\n", m32, std::log2(m32));
  CK(hipFree(dv));
  CK(hipFree(e64));
  CK(hipFree(e32));
  CK(hipFree(out));
  return 0;
}
