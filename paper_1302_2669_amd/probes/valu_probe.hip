// VALU throughput probe for gfx950: eight independent dependency chains of
// one instruction kind per lane, timed with hip events; shader clock from
// s_memtime against s_memrealtime (100 MHz).  Supports the integer-ALU peak
// used for the chain kernel's roofline.
//
//   hipcc -O3 --offload-arch=gfx950 -o valu_probe paper_1302_2669_amd/probes/valu_probe.hip
//   ./valu_probe
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>

#define ITERS 2048
#define BLOCKS 4096
#define THREADS 256

template <int KIND>
__global__ void __launch_bounds__(THREADS) probe(uint32_t* out, uint32_t seed) {
  const uint32_t gid = blockIdx.x * THREADS + threadIdx.x;
  uint32_t a[8];
  uint64_t w[8];
  float f[8];
  const uint32_t b = gid * 2654435761u + seed;
  const float fb = (float)(gid & 255) * 1e-7f;
#pragma unroll
  for (int k = 0; k < 8; ++k) { a[k] = gid + k; w[k] = gid ^ (k * 77u); f[k] = (float)k; }
  for (int it = 0; it < ITERS; ++it) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if constexpr (KIND == 0) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[k]) : "v"(b));
        if constexpr (KIND == 1) asm volatile("v_add_u32 %0, %1, %0" : "+v"(a[k]) : "v"(b));
        if constexpr (KIND == 2) asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(w[k]) : "v"(b), "v"(a[k]) : "vcc");
        if constexpr (KIND == 3) asm volatile("v_mul_hi_u32 %0, %1, %0" : "+v"(a[k]) : "v"(b));
        if constexpr (KIND == 4) asm volatile("v_fma_f32 %0, %1, %1, %0" : "+v"(f[k]) : "v"(fb));
        if constexpr (KIND == 5) asm volatile("v_bitop3_b32 %0, %1, %0, %1 bitop3:0x96" : "+v"(a[k]) : "v"(b));
        if constexpr (KIND == 6) asm volatile("v_bfe_u32 %0, %0, 3, 4" : "+v"(a[k]));
        if constexpr (KIND == 7) asm volatile("v_mul_lo_u32 %0, %1, %0" : "+v"(a[k]) : "v"(b));
        if constexpr (KIND == 8) asm volatile("v_lshl_or_b32 %0, %0, 3, %1" : "+v"(a[k]) : "v"(b));
        if constexpr (KIND == 9) asm volatile("v_cndmask_b32 %0, %0, %1, vcc" : "+v"(a[k]) : "v"(b) : "vcc");
      }
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) r ^= a[k] ^ (uint32_t)w[k] ^ (uint32_t)(w[k] >> 32) ^ __float_as_uint(f[k]);
  out[gid] = r;
}

__global__ void clock_probe(unsigned long long* out, uint32_t seed) {
  const unsigned long long t0 = __builtin_amdgcn_s_memtime();
  const unsigned long long r0 = __builtin_amdgcn_s_memrealtime();
  uint32_t a = threadIdx.x + seed;
  for (int i = 0; i < 4000000; ++i) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a) : "v"(seed));
  const unsigned long long t1 = __builtin_amdgcn_s_memtime();
  const unsigned long long r1 = __builtin_amdgcn_s_memrealtime();
  if (threadIdx.x == 0) { out[0] = t1 - t0; out[1] = r1 - r0; out[2] = a; }
}

template <int KIND>
double run(uint32_t* d_out) {
  hipEvent_t e0, e1;
  hipEventCreate(&e0); hipEventCreate(&e1);
  hipLaunchKernelGGL(probe<KIND>, dim3(BLOCKS), dim3(THREADS), 0, 0, d_out, 1u);
  hipEventRecord(e0, 0);
  hipLaunchKernelGGL(probe<KIND>, dim3(BLOCKS), dim3(THREADS), 0, 0, d_out, 2u);
  hipEventRecord(e1, 0);
  hipEventSynchronize(e1);
  float ms = 0; hipEventElapsedTime(&ms, e0, e1);
  const double ops = (double)BLOCKS * THREADS * ITERS * 64.0;
  return ops / (ms * 1e-3);
}

int main() {
  uint32_t* d_out; unsigned long long* d_clk;
  hipMalloc(&d_out, sizeof(uint32_t) * BLOCKS * THREADS);
  hipMalloc(&d_clk, 3 * sizeof(unsigned long long));
  hipLaunchKernelGGL(clock_probe, dim3(1), dim3(64), 0, 0, d_clk, 3u);
  unsigned long long clk[3];
  hipMemcpy(clk, d_clk, sizeof(clk), hipMemcpyDeviceToHost);
  const double f_ghz = (double)clk[0] / (double)clk[1] * 0.1;
  int cus = 0; hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0);
  int clk_khz = 0; hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeClockRate, 0);
  printf("CUs %d, reported max clock %.3f GHz, measured shader clock (1 wave) %.3f GHz\n", cus, clk_khz * 1e-6, f_ghz);
  const char* names[] = {"v_xor_b32", "v_add_u32", "v_mad_u64_u32", "v_mul_hi_u32", "v_fma_f32", "v_bitop3_b32(xor3)", "v_bfe_u32", "v_mul_lo_u32", "v_lshl_or_b32", "v_cndmask_b32"};
  double r[10];
  r[0] = run<0>(d_out); r[1] = run<1>(d_out); r[2] = run<2>(d_out); r[3] = run<3>(d_out);
  r[4] = run<4>(d_out); r[5] = run<5>(d_out); r[6] = run<6>(d_out); r[7] = run<7>(d_out);
  r[8] = run<8>(d_out); r[9] = run<9>(d_out);
  for (int i = 0; i < 10; ++i)
    printf("%-16s %8.2f T lane-instr/s  = %6.1f lanes/clk/CU at 2.4 GHz\n", names[i], r[i] * 1e-12, r[i] / (cus * 2.4e9));
  return 0;
}
