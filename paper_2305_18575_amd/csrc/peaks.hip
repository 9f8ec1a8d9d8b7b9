// Achievable peaks of the operations the search is built from, measured on
// the current device.  The roofline figures of a kernel are read against
// these as well as against the published peaks: a stream copy for HBM
// bandwidth, random table probes (a read, or a read and an atomicMin, at
// pseudo-random 8-byte slots) for the dedup table, and a bitwise AND-OR loop
// for the integer vector ALU.
#include <algorithm>

#include "device_common.h"

namespace rei {
namespace {

// Stream copy with 16-byte loads and stores, grid-stride.
__global__ __launch_bounds__(256) void peak_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                 uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
    dst[i] = src[i];
}

// Random probes of a table of mask + 1 slots: probe i reads the slot at
// mix64(i) (a dedup-table probe: one 8-byte read somewhere in the table, in
// its own 64-byte line unless two probes meet) and, with kAtomic, lowers the
// slot at the other half of the hash with atomicMin (a survivor's claim).
template <bool kAtomic>
__global__ __launch_bounds__(256) void peak_probe(uint64_t* table, uint64_t mask, uint64_t n, uint64_t* sink) {
  uint64_t acc = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    const uint64_t h = mix64(i ^ 0x9e3779b97f4a7c15ull);
    const uint64_t v = table[h & mask];
    acc ^= v;
    if (kAtomic) atomicMin((unsigned long long*)&table[(h >> 29) & mask], (unsigned long long)(v ^ h));
  }
  if (acc == 0x0123456789abcdefull) sink[0] = acc;  // keeps the loads; never true for the fill value
}

// Bitwise loop: eight independent chains of a = (a & b) | c per step, each
// one fused AND-OR instruction (two 32-bit bitwise operations), b and c
// taken from the other chains.  Written as one VALU instruction per step
// (register operands only, no memory access): the same expression in C++ is
// collapsed by the compiler, since AND and OR are idempotent and the chains
// converge.
constexpr int kChains = 8;
constexpr int kUnroll = 8;

__device__ __forceinline__ uint32_t and_or(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm volatile("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

__global__ __launch_bounds__(256) void peak_bitwise(uint32_t iters, uint32_t seed, uint32_t* sink) {
  const uint32_t t = (uint32_t)(blockIdx.x * 256 + threadIdx.x);
  uint32_t a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = (seed + t) * (2654435761u + 2u * (uint32_t)k);
  for (uint32_t it = 0; it < iters; it += kUnroll) {  // iters: a multiple of kUnroll
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
      for (int k = 0; k < kChains; ++k) a[k] = and_or(a[k], a[(k + 3) % kChains], a[(k + 5) % kChains]);
    }
  }
  uint32_t x = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) x ^= a[k];
  if (x == seed) sink[t & 1023] = x;
}

__global__ void peak_fill(uint64_t* p, uint64_t n, uint64_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

}  // namespace

hipError_t measure_peak(int kind, uint64_t size, double* rate, double* seconds) {
  int dev = 0, cus = 256;
  hipError_t e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  hipStream_t s = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  void* buf = nullptr;
  void* buf2 = nullptr;
  uint64_t* sink = nullptr;
  double best = 1e300, work = 0;
  auto cleanup = [&]() {
    if (s) (void)hipStreamSynchronize(s);
    if (buf) (void)hipFree(buf);
    if (buf2) (void)hipFree(buf2);
    if (sink) (void)hipFree(sink);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (s) (void)hipStreamDestroy(s);
  };
#define PK(call)              \
  do {                        \
    if ((e = (call)) != hipSuccess) { \
      cleanup();              \
      return e;               \
    }                         \
  } while (0)
  PK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  PK(hipEventCreate(&a));
  PK(hipEventCreate(&b));
  PK(hipMalloc(&sink, 4096 * sizeof(uint64_t)));
  const dim3 grid((uint32_t)cus * 8), block(256);
  auto timed = [&](auto&& launch) -> hipError_t {
    hipError_t r;
    for (int rep = 0; rep < 6; ++rep) {  // the first is a warm-up
      if ((r = hipEventRecord(a, s)) != hipSuccess) return r;
      launch();
      if ((r = hipGetLastError()) != hipSuccess) return r;
      if ((r = hipEventRecord(b, s)) != hipSuccess) return r;
      if ((r = hipEventSynchronize(b)) != hipSuccess) return r;
      float ms = 0;
      if ((r = hipEventElapsedTime(&ms, a, b)) != hipSuccess) return r;
      if (rep) best = std::min(best, (double)ms * 1e-3);
    }
    return hipSuccess;
  };
  if (kind == 0) {  // copy: size bytes read and size bytes written
    const uint64_t n = std::max<uint64_t>(1, size / 16);
    PK(hipMalloc(&buf, n * 16));
    PK(hipMalloc(&buf2, n * 16));
    hipLaunchKernelGGL(peak_fill, grid, block, 0, s, (uint64_t*)buf, n * 2, 1ull);
    PK(timed([&] { hipLaunchKernelGGL(peak_copy, grid, block, 0, s, (const uint4*)buf, (uint4*)buf2, n); }));
    work = 2.0 * (double)n * 16;
  } else if (kind == 1 || kind == 2) {  // probes of a table of size bytes (a power of two)
    uint64_t slots = 1;
    while (slots * 2 * 8 <= std::max<uint64_t>(size, 8)) slots *= 2;
    const uint64_t probes = 1ull << 27;
    PK(hipMalloc(&buf, slots * 8));
    hipLaunchKernelGGL(peak_fill, grid, block, 0, s, (uint64_t*)buf, slots, ~0ull);
    if (kind == 1)
      PK(timed([&] { hipLaunchKernelGGL(peak_probe<false>, grid, block, 0, s, (uint64_t*)buf, slots - 1, probes, sink); }));
    else
      PK(timed([&] { hipLaunchKernelGGL(peak_probe<true>, grid, block, 0, s, (uint64_t*)buf, slots - 1, probes, sink); }));
    work = (double)probes;
  } else if (kind == 3) {  // bitwise: 32-bit lane operations
    const uint32_t iters = 1u << 14;
    PK(timed([&] { hipLaunchKernelGGL(peak_bitwise, grid, block, 0, s, iters, 7u, (uint32_t*)sink); }));
    work = (double)grid.x * 256 * iters * kChains * 2;
  } else {
    cleanup();
    return hipErrorInvalidValue;
  }
#undef PK
  cleanup();
  *seconds = best;
  *rate = work / best;
  return hipSuccess;
}

}  // namespace rei
