// tpmc_ceilings.hip -- microkernels that measure the ceilings of the path's
// roofline on the device it runs on: VALU issue (FP32 and FP64 FMA, int32
// multiply-add), streaming reads from L2, the Infinity Cache or HBM (the
// buffer's size decides which), and int64 atomic adds in global memory and in
// LDS.  The seeding, traversal and tally kernels are bound by these rather
// than by HBM, so the measured values put the published peaks into context.
//
// Every kernel keeps its result live through a store that only a launch with
// a one-thread workgroup would make; the launches below always use 256
// threads, so the sink is never written, but the compiler cannot drop the work.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tpmc_internal.h"
#include "tpmc_launch.h"

namespace tpmc {
namespace {

constexpr int kCeilIlp = 8;  // independent dependency chains per lane

template <class T>
__global__ __launch_bounds__(kBlock) void valu_fma_kernel(T* __restrict__ sink, uint32_t iters, T seed) {
  T a[kCeilIlp];
#pragma unroll
  for (int i = 0; i < kCeilIlp; ++i) a[i] = seed + (T)(threadIdx.x + i);
  const T m = (T)0.999999, c = (T)1e-7;
#pragma unroll 1
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
#pragma unroll
      for (int i = 0; i < kCeilIlp; ++i) a[i] = fma(a[i], m, c);
    }
  }
  T s = 0;
#pragma unroll
  for (int i = 0; i < kCeilIlp; ++i) s += a[i];
  if (blockDim.x == 1) sink[0] = s;
}

__global__ __launch_bounds__(kBlock) void valu_imad_kernel(uint32_t* __restrict__ sink, uint32_t iters, uint32_t seed) {
  uint32_t a[kCeilIlp];
#pragma unroll
  for (int i = 0; i < kCeilIlp; ++i) a[i] = seed + threadIdx.x + (uint32_t)i;
#pragma unroll 1
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
#pragma unroll
      for (int i = 0; i < kCeilIlp; ++i) a[i] = a[i] * a[i] + 0x7F4A7C15u;  // no two steps fold into one
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kCeilIlp; ++i) s ^= a[i];
  if (blockDim.x == 1) sink[0] = s;
}

// Grid-stride reads of 16 bytes per lane, `passes` times over the buffer.
__global__ __launch_bounds__(kBlock) void read_kernel(const uint4* __restrict__ p, uint64_t n16, uint32_t passes,
                                                      uint32_t* __restrict__ sink) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t start = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
#pragma unroll 1
  for (uint32_t pass = 0; pass < passes; ++pass) {
    uint64_t i = start;
    for (; i + 3 * stride < n16; i += 4 * stride) {  // four loads in flight per lane
      const uint4 v0 = p[i], v1 = p[i + stride], v2 = p[i + 2 * stride], v3 = p[i + 3 * stride];
      acc ^= (v0.x ^ v0.y ^ v0.z ^ v0.w) ^ (v1.x ^ v1.y ^ v1.z ^ v1.w) ^ (v2.x ^ v2.y ^ v2.z ^ v2.w) ^
             (v3.x ^ v3.y ^ v3.z ^ v3.w);
    }
    for (; i < n16; i += stride) {
      const uint4 v = p[i];
      acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
  }
  if (blockDim.x == 1) sink[0] = acc;
}

// per_thread int64 atomic adds per lane into slots addresses (slots = 1: all
// lanes of the grid on one address).
__global__ __launch_bounds__(kBlock) void atomic_i64_kernel(unsigned long long* __restrict__ p, uint32_t slots,
                                                            uint32_t per_thread) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll 1
  for (uint32_t k = 0; k < per_thread; ++k) {
    const uint32_t idx = (gid * 0x9E3779B1u + k * 0x85EBCA77u) % slots;
    atomicAdd(p + idx, 1ull);
  }
}

__global__ __launch_bounds__(kBlock) void lds_atomic_i64_kernel(unsigned long long* __restrict__ sink, uint32_t slots,
                                                                uint32_t per_thread) {
  __shared__ unsigned long long s[1024];
  for (uint32_t i = threadIdx.x; i < 1024; i += blockDim.x) s[i] = 0;
  __syncthreads();
#pragma unroll 1
  for (uint32_t k = 0; k < per_thread; ++k) {
    const uint32_t idx = (threadIdx.x * 0x9E3779B1u + k * 0x85EBCA77u) % slots;
    atomicAdd(s + idx, 1ull);
  }
  __syncthreads();
  const unsigned long long v = s[threadIdx.x % slots];
  if (blockDim.x == 1) sink[0] = v;
}

}  // namespace

void launch_ceiling_valu(uint32_t kind, int grid, uint32_t iters, void* sink, hipStream_t st) {
  if (kind == 0) valu_fma_kernel<float><<<grid, kBlock, 0, st>>>(static_cast<float*>(sink), iters, 1.0f);
  else if (kind == 1) valu_fma_kernel<double><<<grid, kBlock, 0, st>>>(static_cast<double*>(sink), iters, 1.0);
  else valu_imad_kernel<<<grid, kBlock, 0, st>>>(static_cast<uint32_t*>(sink), iters, 1u);
}

uint64_t ceiling_valu_ops_per_lane(uint32_t iters) { return (uint64_t)iters * 16u * kCeilIlp; }

void launch_ceiling_read(const void* p, uint64_t bytes, uint32_t passes, int grid, hipStream_t st) {
  read_kernel<<<grid, kBlock, 0, st>>>(static_cast<const uint4*>(p), bytes / 16, passes,
                                       static_cast<uint32_t*>(const_cast<void*>(p)));
}

void launch_ceiling_atomic(void* p, uint32_t slots, uint32_t per_thread, int grid, hipStream_t st) {
  atomic_i64_kernel<<<grid, kBlock, 0, st>>>(static_cast<unsigned long long*>(p), slots, per_thread);
}

void launch_ceiling_lds_atomic(void* sink, uint32_t slots, uint32_t per_thread, int grid, hipStream_t st) {
  lds_atomic_i64_kernel<<<grid, kBlock, 0, st>>>(static_cast<unsigned long long*>(sink), slots, per_thread);
}

}  // namespace tpmc
