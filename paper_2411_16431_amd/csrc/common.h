// Internal helpers of libtnbb: error plumbing, device buffers, bit tricks.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <string>
#include <utility>
#include <vector>

#include "tnbb.h"

namespace tnb {

struct Error {
  tnb_status code;
  std::string msg;
};

[[noreturn]] inline void fail(tnb_status code, const std::string& msg) { throw Error{code, msg}; }

inline void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) fail(TNB_ENOMEM, std::string(what) + ": out of device memory");
    fail(TNB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}
#define TNB_STR2(x) #x
#define TNB_STR(x) TNB_STR2(x)
#define HIPC(x) ::tnb::hip_check((x), #x " [" __FILE__ ":" TNB_STR(__LINE__) "]")

void set_error(const std::string& msg);
void clear_error();

// Device memory of the library: hipMalloc/hipFree, or the caller's
// allocator when one is installed (tnb_set_allocator).  A block is returned
// to the allocator that gave it.
struct Allocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*release)(void*, void*) = nullptr;
  void* user = nullptr;
};
const Allocator* current_allocator();  // nullptr: hipMalloc / hipFree
void* dev_alloc(size_t bytes, const Allocator** owner);
void dev_free(void* p, const Allocator* owner);

// Launch-variant autotuner (tnb_autotune): runs run(v) for the stored, or
// (when measuring) the fastest, of n variants of `key`; returns the choice.
int autotune_pick(const std::string& key, int n, const std::function<void(int)>& run, hipStream_t st);

// Owning device allocation, freed on destruction.  With hipFree the runtime
// waits for the device; a caller's allocator must order reuse after the
// work queued on the library's streams (a stream-ordered caching allocator
// on the same stream does).
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  const Allocator* owner = nullptr;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), owner(o.owner) { o.p = nullptr; o.n = 0; o.owner = nullptr; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      owner = o.owner;
      o.p = nullptr;
      o.n = 0;
      o.owner = nullptr;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    n = count;
    if (count) p = static_cast<T*>(dev_alloc(count * sizeof(T), &owner));
  }
  void release() {
    if (p) dev_free(p, owner);
    p = nullptr;
    n = 0;
    owner = nullptr;
  }
  void upload(const T* host, size_t count, hipStream_t s) {
    if (count > n) alloc(count);
    if (count) HIPC(hipMemcpyAsync(p, host, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void upload(const std::vector<T>& v, hipStream_t s) { upload(v.data(), v.size(), s); }
};

inline int popcount32(uint32_t m) { return __builtin_popcount(m); }

// pext on the host (bits of x selected by mask, packed to the low end).
inline uint32_t pext_host(uint32_t x, uint32_t mask) {
  uint32_t out = 0;
  int j = 0;
  for (int b = 0; b < 32; ++b)
    if (mask >> b & 1u) out |= ((x >> b) & 1u) << j++;
  return out;
}
inline uint32_t pdep_host(uint32_t y, uint32_t mask) {
  uint32_t out = 0;
  int j = 0;
  for (int b = 0; b < 32; ++b)
    if (mask >> b & 1u) out |= ((y >> j++) & 1u) << b;
  return out;
}

__device__ __forceinline__ uint32_t pext_dev(uint32_t x, uint32_t mask) {
  uint32_t out = 0;
  int j = 0;
  while (mask) {
    int b = __builtin_ctz(mask);
    out |= ((x >> b) & 1u) << j++;
    mask &= mask - 1u;
  }
  return out;
}
__device__ __forceinline__ uint32_t pdep_dev(uint32_t y, uint32_t mask) {
  uint32_t out = 0;
  int j = 0;
  while (mask) {
    int b = __builtin_ctz(mask);
    out |= ((y >> j++) & 1u) << b;
    mask &= mask - 1u;
  }
  return out;
}

// Validated host copy of an instance plus its cluster bookkeeping.
struct Lattice {
  int N = 0, E = 0, R = 0, C = 0;
  std::vector<int32_t> ei, ej, cell_of;
  std::vector<double> J, h;
  std::vector<std::vector<int>> spins;  // per cell, ascending
  std::vector<int> bit;                 // bit position of a spin in its cell
  std::vector<int> k;                   // spins per cell
  int cells() const { return R * C; }
  int cell(int r, int c) const { return (r >= 0 && r < R && c >= 0 && c < C) ? r * C + c : -1; }
};

Lattice validate_instance(const tnb_instance* inst);

// A device weight of 1 for the current device (a constant of the code
// object, looked up once per device).
const double* unit_weight();
const float* unit_weight32();

template <class F>
tnb_status guarded(F&& f) {
  try {
    clear_error();
    f();
    return TNB_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return TNB_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return TNB_EDEVICE;
  } catch (...) {
    set_error("unknown failure");
    return TNB_EDEVICE;
  }
}

// Optional per-kernel timing with HIP events recorded on the launch stream.
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
  double flops, bytes;
};
bool prof_on();
void prof_push(const ProfRec& r);
// A timing event of the current device from a pool that is filled when
// profiling is switched on, so that timed regions create no events.
hipEvent_t prof_event();
struct KTimer {
  bool on;
  ProfRec r;
  hipStream_t st;
  KTimer(const char* name, hipStream_t s, double flops, double bytes) : on(prof_on()), st(s) {
    r = ProfRec{name, nullptr, nullptr, flops, bytes};
    if (on) {
      r.a = prof_event();
      r.b = prof_event();
      HIPC(hipEventRecord(r.a, st));
    }
  }
  ~KTimer() {
    if (on) {
      (void)hipEventRecord(r.b, st);
      prof_push(r);
    }
  }
};

enum HandleKind : uint32_t { KIND_CLUSTERS = 0x544E4231u, KIND_ENV = 0x544E4232u, KIND_BEAM = 0x544E4233u };

}  // namespace tnb
