// probe.hip -- microbenchmarks of the device rates the dedispersion kernel
// is measured against: the vector instructions it is made of (32-bit add,
// three-input add, byte permute) and LDS reads (16-byte and 4-byte).  Each rate is what the
// device sustains at its actual clock, in lane-operations (or bytes) per
// second, so a kernel's fraction can be stated against the instruction mix
// it issues as well as against the figures derived from unit counts.  On
// MI355X two-operand 32-bit ops issue at two lane-ops per lane per clock and
// three-operand ops (v_add3_u32, v_perm_b32) at one.
#include "sps_internal.h"

namespace sps {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeBlocks = 8192;  // 4 rounds of 8 workgroups on each of 256 CUs
constexpr int kAddUnroll = 16;
constexpr int kAddChains = 8;

// Eight independent chains of one instruction per lane, kAddUnroll deep per
// iteration, in inline asm so that the compiler can neither fold nor drop
// them.  OP 0: v_add_u32 (two operands); 1: v_add3_u32 (three operands);
// 2: v_perm_b32 (byte select, the dedispersion kernel's realignment).
template <int OP>
__global__ __launch_bounds__(kProbeThreads) void valu_probe_kernel(uint32_t *__restrict__ out,
                                                                   int iters) {
  const uint32_t b = threadIdx.x | 1u, c = 0x0C020C00u + (threadIdx.x & 3u) * 0x10001u;
  uint32_t a0 = threadIdx.x, a1 = a0 + 1u, a2 = a0 + 2u, a3 = a0 + 3u;
  uint32_t a4 = a0 + 4u, a5 = a0 + 5u, a6 = a0 + 6u, a7 = a0 + 7u;
#define SPS_PROBE_CHAINS(I)                                                                  \
  asm volatile(I(0) I(1) I(2) I(3) I(4) I(5) I(6) I(7)                                       \
               : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7) \
               : "v"(b), "v"(c))
#define SPS_ADD(k) "v_add_u32 %" #k ", %" #k ", %8\n\t"
#define SPS_ADD3(k) "v_add3_u32 %" #k ", %" #k ", %8, %9\n\t"
#define SPS_PERM(k) "v_perm_b32 %" #k ", %" #k ", %8, %9\n\t"
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kAddUnroll; ++u) {
      if constexpr (OP == 0) SPS_PROBE_CHAINS(SPS_ADD);
      if constexpr (OP == 1) SPS_PROBE_CHAINS(SPS_ADD3);
      if constexpr (OP == 2) SPS_PROBE_CHAINS(SPS_PERM);
    }
  }
#undef SPS_ADD
#undef SPS_ADD3
#undef SPS_PERM
#undef SPS_PROBE_CHAINS
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}

// 16-byte LDS reads, lane-consecutive (conflict-free), four per iteration.
// Which half of the buffer an iteration reads depends on the running sum, so
// the reads can be neither hoisted nor folded (a loop-invariant address
// lets the compiler lift them out of the loop); two three-input adds per
// component keep the vector work under the LDS time.
__global__ __launch_bounds__(kProbeThreads) void lds_read_probe_kernel(uint32_t *__restrict__ out,
                                                                       int iters) {
  __shared__ u32x4 buf[8 * kProbeThreads];  // 32 KB
  for (int i = threadIdx.x; i < 8 * kProbeThreads; i += kProbeThreads)
    buf[i] = u32x4{(uint32_t)i, (uint32_t)i + 1u, (uint32_t)i + 2u, (uint32_t)i + 3u};
  __syncthreads();
  u32x4 acc = {0u, 0u, 0u, 0u};
  for (int i = 0; i < iters; ++i) {
    const u32x4 *p = buf + (acc.x & 1u) * (4 * kProbeThreads) + threadIdx.x;
    const u32x4 v0 = p[0], v1 = p[kProbeThreads], v2 = p[2 * kProbeThreads],
                v3 = p[3 * kProbeThreads];
    acc = acc + v0 + v1;
    acc = acc + v2 + v3;
  }
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

// 4-byte LDS reads, lane-consecutive (conflict-free), eight per iteration:
// the access width of the dedispersion kernel's window reads.  The address
// depends on the running sum as above.
__global__ __launch_bounds__(kProbeThreads) void lds_read32_probe_kernel(uint32_t *__restrict__ out,
                                                                         int iters) {
  __shared__ uint32_t buf[16 * kProbeThreads];  // 16 KB
  for (int i = threadIdx.x; i < 16 * kProbeThreads; i += kProbeThreads) buf[i] = (uint32_t)i;
  __syncthreads();
  uint32_t acc = 0u, acc2 = 0u;
  for (int i = 0; i < iters; ++i) {
    const uint32_t *p = buf + (acc & 1u) * (8 * kProbeThreads) + threadIdx.x;
    const uint32_t v0 = p[0], v1 = p[kProbeThreads], v2 = p[2 * kProbeThreads],
                   v3 = p[3 * kProbeThreads], v4 = p[4 * kProbeThreads], v5 = p[5 * kProbeThreads],
                   v6 = p[6 * kProbeThreads], v7 = p[7 * kProbeThreads];
    acc = acc + v0 + v1;
    acc2 = acc2 + v2 + v3;
    acc = acc + v4 + v5;
    acc2 = acc2 + v6 + v7;
  }
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = acc ^ acc2;
}

// Mean duration of one launch (ms), after an untimed shorter one.
template <typename F>
hipError_t time_launch(F launch, hipEvent_t e0, hipEvent_t e1, hipStream_t stream, float *ms) {
  launch(true);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(e0, stream);
  if (e == hipSuccess) {
    launch(false);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  if (e == hipSuccess && *ms <= 0.0f) e = hipErrorUnknown;
  return e;
}

}  // namespace

hipError_t probe_device_peaks(double *rates, hipStream_t stream) {
  constexpr int kAddIters = 1000, kLdsIters = 4000;
  uint32_t *out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&out, sizeof(uint32_t) * (size_t)kProbeBlocks * kProbeThreads);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const double threads = (double)kProbeBlocks * kProbeThreads;
  const dim3 grid(kProbeBlocks), block(kProbeThreads);
  float ms = 0.0f;
  auto valu = [&](auto kern, int slot) {
    if (e != hipSuccess) return;
    e = time_launch([&](bool warm) {
      hipLaunchKernelGGL(kern, grid, block, 0, stream, out, warm ? kAddIters / 10 : kAddIters);
    }, e0, e1, stream, &ms);
    if (e == hipSuccess) rates[slot] = threads * kAddIters * kAddUnroll * kAddChains / (ms * 1e-3);
  };
  valu(valu_probe_kernel<0>, 0);
  valu(valu_probe_kernel<1>, 1);
  valu(valu_probe_kernel<2>, 2);
  if (e == hipSuccess) {
    e = time_launch([&](bool warm) {
      hipLaunchKernelGGL(lds_read_probe_kernel, grid, block, 0, stream, out,
                         warm ? kLdsIters / 10 : kLdsIters);
    }, e0, e1, stream, &ms);
    if (e == hipSuccess) rates[3] = threads * kLdsIters * 4.0 * 16.0 / (ms * 1e-3);
  }
  if (e == hipSuccess) {
    e = time_launch([&](bool warm) {
      hipLaunchKernelGGL(lds_read32_probe_kernel, grid, block, 0, stream, out,
                         warm ? kLdsIters / 10 : kLdsIters);
    }, e0, e1, stream, &ms);
    if (e == hipSuccess) rates[4] = threads * kLdsIters * 8.0 * 4.0 / (ms * 1e-3);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (out) (void)hipFree(out);
  return e;
}

}  // namespace sps
