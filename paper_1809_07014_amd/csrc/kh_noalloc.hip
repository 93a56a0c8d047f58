// kh_count_noalloc: kh_count for callers that cannot allocate device memory.
//
// Every device block the pipeline needs (packed planes, counters, Bloom
// filter, sighting bits, hash table, classify output, sort buffers, heavy
// hitter entries) is carved, in stack order, from one file-scope device
// array of KH_NOALLOC_SCRATCH_BYTES.  Each device holds its own copy of the
// array (it is part of the code object loaded there) until the process
// ends; its device address is looked up once per device, with that device
// current, and only that address is ever handed to kernels or copies (the
// array's name in host code is a host-side stand-in, not a device address).
// The rows go straight to the caller's buffers.  Nothing is allocated or
// freed on the device; the kernels and the pipeline are kh_count's own.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kh_host.hpp"

using namespace kh;

namespace {

constexpr uint64_t kScratchBytes = KH_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// Per device: the array's device address (looked up once) and a lock that
// serialises the calls (they share the array).
std::mutex g_mu[kMaxDevices];
uint8_t* g_scratch[kMaxDevices] = {};

int scratch_of(int device, uint8_t** out) {
  if (!g_scratch[device]) {
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return fail(KH_EDEVICE, "device %d is %s; this library is built for gfx950", device,
                  prop.gcnArchName);
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(KH_EDEVICE, "no device address for the scratch array");
    g_scratch[device] = static_cast<uint8_t*>(ptr);
  }
  *out = g_scratch[device];
  return KH_OK;
}

}  // namespace

extern "C" int kh_count_noalloc(const kh_reads* reads, const kh_params* params, void* stream,
                                uint64_t* keys, uint32_t* counts, uint32_t* ext,
                                uint8_t* codes, int64_t max_rows, int64_t* n_rows,
                                uint64_t* n_windows) {
  if (n_rows) *n_rows = 0;
  if (n_windows) *n_windows = 0;
  if (!reads || !n_rows) return fail(KH_EINVAL, "reads or n_rows is NULL");
  KH_TRY(check_params(params));
  if (reads->n_reads < 0) return fail(KH_EINVAL, "n_reads < 0");
  if (reads->n_reads > 0 && !reads->on_device)
    return fail(KH_EINVAL, "kh_count_noalloc takes reads in device memory (on_device = 1)");
  if (reads->n_reads > 0 && (!reads->offsets || !reads->seq || !reads->qual))
    return fail(KH_EINVAL, "seq, qual or offsets is NULL");
  if (max_rows < 0) return fail(KH_EINVAL, "max_rows < 0");
  if (max_rows > 0 && (!keys || !counts || !ext || !codes))
    return fail(KH_EINVAL, "an output buffer is NULL");
  int device = 0;
  HIP_TRY(hipGetDevice(&device));
  if (device < 0 || device >= kMaxDevices)
    return fail(KH_EINVAL, "device %d out of range", device);
  hipStream_t s = static_cast<hipStream_t>(stream);

  std::lock_guard<std::mutex> lk(g_mu[device]);
  uint8_t* base = nullptr;
  KH_TRY(scratch_of(device, &base));
  if (reads->n_reads > 0) {  // the input bound, before anything is launched
    int64_t n = 0;
    HIP_TRY(hipMemcpyAsync(&n, reads->offsets + reads->n_reads, sizeof n,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (n > (int64_t)KH_NOALLOC_MAX_BASES)
      return fail(KH_EINVAL, "%lld bases exceed the no-allocation limit of %llu",
                  (long long)n, (unsigned long long)KH_NOALLOC_MAX_BASES);
  }

  // A context on the stack whose pool carves the scratch array: counters
  // first, then whatever the pipeline asks for.
  kh_ctx ctx;
  ctx.device = device;
  ctx.pool.device = device;
  ctx.pool.arena = base;
  ctx.pool.arena_size = kScratchBytes;
  kh_default_tuning(&ctx.tune);
  void* c = nullptr;
  KH_TRY(ctx.pool.get(&c, sizeof(uint64_t) * kCtrCount));
  ctx.ctr = static_cast<unsigned long long*>(c);

  kh_table t;
  t.k = params->k;
  t.W = (params->k + 31) / 32;
  t.dst_keys = keys;
  t.dst_counts = counts;
  t.dst_ext = ext;
  t.dst_codes = codes;
  t.dst_cap = max_rows;
  const int rc = count_into(&ctx, reads, *params, s, &t);
  *n_rows = t.n_rows;
  if (n_windows) *n_windows = t.n_windows;
  if (rc != KH_OK) {
    // every launch of this call has finished before the next call may
    // reuse the array
    (void)hipStreamSynchronize(s);
  }
  return rc;
}
