// Roofline microbenchmarks for the k-mer analysis kernels on MI355X.
//
// Measures the ceilings the counting passes run against: streaming copy and
// read-only streaming bandwidth, random 8-byte gathers (independent and dependent pairs), random
// device-scope atomics (add, returning or, CAS) over buffers from 4 MB (L2)
// to 32 GB (HBM), and the table-slot pattern (one key load plus three atomics
// in one 32- or 64-byte slot).  With the argument "pmc" it runs one launch of
// the copy, read, gather, atomic and slot kernels only, for hardware-counter runs
// (the copy kernel moves a known 8 GiB read + 8 GiB write and calibrates the
// FETCH_SIZE / WRITE_SIZE counters).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CK(x)                                                              \
  do {                                                                     \
    hipError_t e = (x);                                                    \
    if (e != hipSuccess) {                                                 \
      std::printf("error: %s: %s\n", #x, hipGetErrorString(e));            \
      std::exit(1);                                                        \
    }                                                                      \
  } while (0)

__device__ __forceinline__ uint64_t mix(uint64_t x) {  // MurmurHash3 fmix64
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

__global__ void k_copy(const uint4* __restrict__ a, uint4* __restrict__ b,
                       uint64_t n) {
  const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += st)
    b[i] = a[i];
}

// Read-only stream: every 16-byte word of the buffer is loaded once, four
// loads in flight per thread; the sum is written only if it equals a
// sentinel, which keeps the loads.
__global__ void k_read(const uint4* __restrict__ a, uint64_t n, uint64_t* __restrict__ sink) {
  const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  uint64_t acc = 0;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * st < n; i += 4 * st) {
    const uint4 v0 = a[i], v1 = a[i + st], v2 = a[i + 2 * st], v3 = a[i + 3 * st];
    acc += (uint64_t)v0.x + v0.y + v0.z + v0.w + v1.x + v1.y + v1.z + v1.w;
    acc += (uint64_t)v2.x + v2.y + v2.z + v2.w + v3.x + v3.y + v3.z + v3.w;
  }
  for (; i < n; i += st) {
    const uint4 v = a[i];
    acc += (uint64_t)v.x + v.y + v.z + v.w;
  }
  if (acc == 0x1234567) sink[0] = acc;
}

enum Mode { GATHER, GATHER_DEP2, ADD32, ADD64, OR64_RET, CAS64, SLOT32, SLOT64, NMODES };
static const char* kNames[NMODES] = {"gather8", "gather8_dependent_pair",
                                     "atomic_add_u32", "atomic_add_u64",
                                     "atomic_or_u64_returning", "atomic_cas_u64",
                                     "slot32_load_3atomics", "slot64_load_3atomics"};

// Every index is hash(i) scaled into [0, nwords): all accesses are in bounds.
__global__ void k_rand(uint64_t* __restrict__ t, uint64_t nwords, uint64_t nops,
                       int mode, uint64_t* __restrict__ sink) {
  const uint64_t st = (uint64_t)gridDim.x * blockDim.x;
  uint64_t acc = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nops; i += st) {
    const uint64_t h = mix(i * 0x9e3779b97f4a7c15ull + 12345);
    const uint64_t w = __umul64hi(h, nwords);
    switch (mode) {
      case GATHER: acc += t[w]; break;
      case GATHER_DEP2: {
        const uint64_t v = t[w];
        acc += t[__umul64hi(mix(h ^ v), nwords)];
        break;
      }
      case ADD32:
        __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(t) + __umul64hi(h, 2 * nwords), 1u,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      case ADD64:
        __hip_atomic_fetch_add(t + w, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      case OR64_RET:
        acc += __hip_atomic_fetch_or(t + w, 1ull << (h & 63), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
        break;
      case CAS64: {
        uint64_t e = 0;
        __hip_atomic_compare_exchange_strong(t + w, &e, h | 1, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        acc += e;
        break;
      }
      default: {  // SLOT32 / SLOT64
        const uint64_t words = mode == SLOT32 ? 4 : 8;
        uint64_t* s = t + __umul64hi(h, nwords / words) * words;
        acc += s[0];
        __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(s + 1), 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(s + 2, 1ull << (16 * (h & 3)), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(s + 3, 1ull << (16 * ((h >> 2) & 3)), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  if (acc == 0x1234567) sink[0] = acc;  // keeps the loads alive
}

int main(int argc, char** argv) {
  const bool pmc = argc > 1 && argv[1][0] == 'p';
  hipDeviceProp_t p;
  CK(hipGetDeviceProperties(&p, 0));
  std::printf("device %s CUs=%d L2=%d MB clock=%d MHz memory=%.1f GB\n",
              p.gcnArchName, p.multiProcessorCount, p.l2CacheSize >> 20,
              p.clockRate / 1000, p.totalGlobalMem / 1e9);
  hipEvent_t a, b;
  CK(hipEventCreate(&a));
  CK(hipEventCreate(&b));
  uint64_t* sink;
  CK(hipMalloc(&sink, 64));
  {
    const uint64_t bytes = 8ull << 30;
    uint4 *x, *y;
    CK(hipMalloc(&x, bytes));
    CK(hipMalloc(&y, bytes));
    CK(hipMemset(x, 1, bytes));
    CK(hipMemset(y, 0, bytes));
    for (int grid : {1024, 4096, 16384}) {
      if (pmc && grid != 1024) continue;
      float best = 1e30f;
      for (int rep = pmc ? 1 : 0; rep < 3; ++rep) {
        CK(hipEventRecord(a));
        hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, 0, x, y, bytes / 16);
        CK(hipEventRecord(b));
        CK(hipEventSynchronize(b));
        float ms;
        CK(hipEventElapsedTime(&ms, a, b));
        if (rep && ms < best) best = ms;
      }
      std::printf("copy grid=%-6d %8.3f ms  %7.1f GB/s (8 GiB read + 8 GiB write)\n",
                  grid, best, 2.0 * bytes / best / 1e6);
    }
    for (int grid : {1024, 4096, 16384}) {
      if (pmc && grid != 1024) continue;
      float best = 1e30f;
      for (int rep = pmc ? 1 : 0; rep < 3; ++rep) {
        CK(hipEventRecord(a));
        hipLaunchKernelGGL(k_read, dim3(grid), dim3(256), 0, 0, x, bytes / 16, sink);
        CK(hipEventRecord(b));
        CK(hipEventSynchronize(b));
        float ms;
        CK(hipEventElapsedTime(&ms, a, b));
        if (rep && ms < best) best = ms;
      }
      std::printf("read grid=%-6d %8.3f ms  %7.1f GB/s (8 GiB read)\n", grid, best,
                  1.0 * bytes / best / 1e6);
    }
    CK(hipFree(x));
    CK(hipFree(y));
  }
  const uint64_t sizes[] = {4ull << 20, 64ull << 20, 256ull << 20, 1ull << 30,
                            8ull << 30, 32ull << 30};
  uint64_t* t;
  CK(hipMalloc(&t, 32ull << 30));
  CK(hipMemset(t, 0, 32ull << 30));
  const uint64_t nops = 1ull << 28;
  for (int mode = 0; mode < NMODES; ++mode) {
    if (pmc && !(mode == GATHER || mode == ADD64 || mode == SLOT32)) continue;
    for (uint64_t S : sizes) {
      if (pmc && S != (32ull << 30)) continue;
      float best = 1e30f;
      for (int rep = pmc ? 2 : 0; rep < 3; ++rep) {
        CK(hipEventRecord(a));
        hipLaunchKernelGGL(k_rand, dim3(16384), dim3(256), 0, 0, t, S / 8, nops, mode, sink);
        CK(hipEventRecord(b));
        CK(hipEventSynchronize(b));
        float ms;
        CK(hipEventElapsedTime(&ms, a, b));
        if (rep && ms < best) best = ms;
      }
      std::printf("%-24s buffer=%8.0f MB  %8.3f ms  %.3e ops/s\n", kNames[mode],
                  S / 1048576.0, best, nops / (best * 1e-3));
    }
  }
  CK(hipFree(t));
  std::printf("done\n");
  return 0;
}
