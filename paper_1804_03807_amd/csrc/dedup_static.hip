// The duplicate-endpoint scan (dedup.hip's kernels) in a workspace the
// library holds per GPU, for callers that cannot allocate device memory: a
// file-scope __device__ array, so each GPU the library runs on has its own
// copy for the life of the process.  In host code the array's name is only a
// stand-in; its device address is looked up once per device (with that
// device current) and kept.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "hp_internal.hpp"

namespace hp {
namespace {

constexpr long long kStaticMaxConverged = 1ll << 19;
constexpr size_t kStaticArrays = (size_t)kStaticMaxConverged * 4 * 8;  // keys, ids, sorted copies
constexpr size_t kStaticCounters = 256;
constexpr size_t kStaticSortBytes = (size_t)20 << 20;
constexpr size_t kStaticBytes = kStaticArrays + kStaticCounters + kStaticSortBytes;

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

// counters to zero with a kernel (no memset node in a captured graph)
__global__ void k_zero_u64(unsigned long long *p, int count) {
  if ((int)threadIdx.x < count) p[threadIdx.x] = 0ull;
}

std::mutex g_mu;
std::map<int, unsigned char *> g_ptr;  // device -> address of scratch on it

// The device address of `scratch` on `device`, which must be current.
hipError_t scratch_on(int device, unsigned char **out) {
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_ptr.find(device);
  if (it == g_ptr.end()) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = g_ptr.emplace(device, (unsigned char *)ptr).first;
  }
  *out = it->second;
  return hipSuccess;
}

}  // namespace
}  // namespace hp

long long hp_dup_static_max_converged() { return hp::kStaticMaxConverged; }

int hp_dup_static_scan(int device, hp::DupArgs a, long long *n_pairs, std::string &err,
                       void *stream) {
  using namespace hp;
  hipStream_t s = (hipStream_t)stream;
  auto device_error = [&](hipError_t e) {
    err = hipGetErrorString(e);
    return -1;
  };
  unsigned char *p = nullptr;
  hipError_t e = scratch_on(device, &p);
  if (e != hipSuccess) return device_error(e);
  const long long C = kStaticMaxConverged;
  if (hp_dup_sort_temp_bytes(C) > kStaticSortBytes) {
    err = "sort workspace of the static scan too small";
    return -1;
  }
  a.keys = (double *)p;
  a.ids = (long long *)(p + (size_t)C * 8);
  a.keys_sorted = (double *)(p + (size_t)C * 16);
  a.ids_sorted = (long long *)(p + (size_t)C * 24);
  a.cap = C;
  a.count = (unsigned long long *)(p + kStaticArrays);
  a.pair_count = a.count + 1;
  a.temp = p + kStaticArrays + kStaticCounters;
  a.temp_bytes = kStaticSortBytes;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, a.count, 2);
  if ((e = hipGetLastError()) != hipSuccess) return device_error(e);
  if ((e = (hipError_t)hp_launch_dup_project(a, s)) != hipSuccess) return device_error(e);
  unsigned long long cnt[2] = {0, 0};
  if ((e = hipMemcpyAsync(cnt, a.count, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                          s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return device_error(e);
  if ((long long)cnt[0] > C) {
    err = std::to_string(cnt[0]) + " converged endpoints: the static scan holds at most " +
          std::to_string(C);
    return -2;
  }
  const long long m = (long long)cnt[0];
  if ((e = (hipError_t)hp_launch_dup_sort(a, m, s)) != hipSuccess ||
      (e = (hipError_t)hp_launch_dup_scan(a, m, s)) != hipSuccess)
    return device_error(e);
  if ((e = hipMemcpyAsync(&cnt[1], a.pair_count, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                          s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return device_error(e);
  *n_pairs = (long long)cnt[1];
  return 0;
}
