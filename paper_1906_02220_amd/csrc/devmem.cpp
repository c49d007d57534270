// Device allocation of the library's buffers, with the optional poisoning
// and guard bands that expose reads of unwritten memory and writes past the
// ends of a buffer.
#include <cstdio>
#include <vector>

#include "internal.hpp"

namespace ctm {

namespace {

constexpr unsigned char kGuardByte = 0xA5;
std::atomic<long long> g_violations{0};

}  // namespace

std::atomic<int>& poison_allocations() {
  static std::atomic<int> flag{[] {
    const char* v = std::getenv("CTM_POISON_ALLOC");
    return (v && *v && !(v[0] == '0' && v[1] == 0)) ? 1 : 0;
  }()};
  return flag;
}

long long guard_violations() { return g_violations.load(); }

void* debug_malloc(size_t nbytes, bool guarded) {
  void* base = nullptr;
  const size_t total = guarded ? nbytes + 2 * kGuardBytes : nbytes;
  if (hipMalloc(&base, total) != hipSuccess) return nullptr;
  if (!guarded) return base;
  char* user = static_cast<char*>(base) + kGuardBytes;
  // the library's streams do not wait for the null stream: finish here
  if (hipMemset(base, kGuardByte, kGuardBytes) != hipSuccess ||
      hipMemset(user, 0xFF, nbytes) != hipSuccess ||
      hipMemset(user + nbytes, kGuardByte, kGuardBytes) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(base);
    return nullptr;
  }
  return user;
}

void debug_free(void* p, size_t nbytes, bool guarded) {
  if (!guarded) {
    (void)hipFree(p);
    return;
  }
  char* user = static_cast<char*>(p);
  char* base = user - kGuardBytes;
  std::vector<unsigned char> band(kGuardBytes);
  for (int side = 0; side < 2; ++side) {
    const char* at = side == 0 ? base : user + nbytes;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(band.data(), at, kGuardBytes, hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipGetLastError();
      std::fprintf(stderr, "ctm: could not read a guard band of a %zu-byte buffer\n", nbytes);
      ++g_violations;
      continue;
    }
    size_t first = kGuardBytes, last = 0, count = 0;
    for (size_t i = 0; i < kGuardBytes; ++i)
      if (band[i] != kGuardByte) {
        if (first == kGuardBytes) first = i;
        last = i;
        ++count;
      }
    if (count) {
      ++g_violations;
      if (side == 0)
        std::fprintf(stderr,
                     "ctm: %zu bytes written before a %zu-byte buffer, from %zu to %zu bytes "
                     "before its start\n",
                     count, nbytes, kGuardBytes - first, kGuardBytes - last);
      else
        std::fprintf(stderr,
                     "ctm: %zu bytes written past the end of a %zu-byte buffer, at offsets "
                     "%zu..%zu past the end\n",
                     count, nbytes, first, last);
      std::fflush(stderr);
    }
  }
  (void)hipFree(base);
}

}  // namespace ctm
