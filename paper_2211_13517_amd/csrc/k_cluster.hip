// Local-maximum clustering of candidate records.
//
// A strong signal leaves a patch of passing cells (its sidelobes in r and z,
// and the same power seen by several harmonic stages).  Record i is kept when
// no record of the same series within |dR| <= rr and |dj| <= rj has a larger
// Gaussian significance; equal significances go to the smaller (j, R).  The
// neighbourhood lookup uses an open-addressing hash table of the records'
// cells in scratch memory (the caller's, or this file's static array for the
// allocation-free variant): a fill, one insert pass and one probe pass, each
// a plain grid over the records (their number is read on the device).
#include <algorithm>
#include <mutex>

#include "launch.hpp"

namespace fdas {

constexpr unsigned long long kEmpty = ~0ull;

__device__ __forceinline__ unsigned long long cell_key(int series, int j, int R) {
  // R < 2^23 (half-bin cells of a 2^22-bin series), j < 2^12
  return ((unsigned long long)series << 35) | ((unsigned long long)j << 23) | (unsigned long long)R;
}

__device__ __forceinline__ uint32_t cell_slot(unsigned long long key, int log2t) {
  return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - log2t));
}

__global__ void k_cluster_clear(unsigned long long* keys, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    keys[i] = kEmpty;
}

__global__ void k_cluster_insert(const fdas_candidate* __restrict__ c, const unsigned long long* __restrict__ count,
                                 int64_t capacity, unsigned long long* keys, int32_t* idx, int log2t) {
  const int64_t n = min((int64_t)*count, capacity);
  const uint32_t mask = (1u << log2t) - 1u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long key = cell_key(c[i].series, c[i].j, c[i].R);
    uint32_t h = cell_slot(key, log2t);
    // the table has at least twice as many slots as records: an empty slot
    // is always reached
    for (uint32_t probe = 0; probe <= mask; ++probe, h = (h + 1) & mask) {
      const unsigned long long prev = atomicCAS(&keys[h], kEmpty, key);
      if (prev == kEmpty) {
        idx[h] = (int32_t)i;
        break;
      }
      if (prev == key) break;  // one record per cell: cannot happen
    }
  }
}

__global__ void k_cluster_peaks(const fdas_candidate* __restrict__ c, const unsigned long long* __restrict__ count,
                                int64_t capacity, const unsigned long long* __restrict__ keys,
                                const int32_t* __restrict__ idx, int log2t, int rr, int rj, uint8_t* keep) {
  const int64_t n = min((int64_t)*count, capacity);
  const uint32_t mask = (1u << log2t) - 1u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const fdas_candidate me = c[i];
    const unsigned long long mykey = cell_key(me.series, me.j, me.R);
    bool peak = true;
    for (int dj = -rj; dj <= rj && peak; ++dj) {
      for (int dr = -rr; dr <= rr && peak; ++dr) {
        // cells off the key's range hold no record (and must not alias one)
        if ((dj == 0 && dr == 0) || me.j + dj < 0 || me.R + dr < 0 || me.j + dj >= (1 << 12) ||
            me.R + dr >= (1 << 23))
          continue;
        const unsigned long long key = cell_key(me.series, me.j + dj, me.R + dr);
        uint32_t h = cell_slot(key, log2t);
        for (uint32_t probe = 0; probe <= mask; ++probe, h = (h + 1) & mask) {
          const unsigned long long k = keys[h];
          if (k == kEmpty) break;
          if (k == key) {
            const float s = c[idx[h]].sigma;
            if (s > me.sigma || (s == me.sigma && key < mykey)) peak = false;
            break;
          }
        }
      }
    }
    keep[i] = peak ? 1 : 0;
  }
}

int cluster_log2_slots(int64_t capacity) {
  int l = 1;
  while ((1ll << l) < 2 * std::max<int64_t>(capacity, 1)) ++l;
  return l;
}

int64_t cluster_scratch_bytes(int64_t capacity) {
  const int64_t t = 1ll << cluster_log2_slots(capacity);
  return t * (int64_t)sizeof(unsigned long long) + t * (int64_t)sizeof(int32_t);
}

// Scratch of the allocation-free variant: one table for kClusterStaticMaxRecords
// records (2^21 slots of an 8-byte key and a 4-byte index, 24 MiB), a copy
// per GPU that the library runs on, held until the process ends.  Host code
// never passes `scratch` itself to a kernel: its device address comes from
// hipGetSymbolAddress, per device.
constexpr int64_t kClusterStaticBytes = (int64_t(2) << 20) * 12;
__device__ __align__(256) unsigned char scratch[kClusterStaticBytes];

hipError_t cluster_static_scratch(int device, void** ptr) {
  static_assert((int64_t(1) << 21) * 12 == kClusterStaticBytes, "table size");
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* a = nullptr;
    e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    addr[device] = a;
  }
  *ptr = addr[device];
  return hipSuccess;
}

hipError_t launch_cluster(const fdas_candidate* c, const unsigned long long* count, int64_t capacity, int rr, int rj,
                          void* table, uint8_t* keep, int cus, hipStream_t st) {
  const int log2t = cluster_log2_slots(capacity);
  const int64_t t = 1ll << log2t;
  auto* keys = reinterpret_cast<unsigned long long*>(table);
  auto* idx = reinterpret_cast<int32_t*>(keys + t);
  const int grid_t = (int)std::min<int64_t>((t + 255) / 256, (int64_t)cus * 8);
  const int grid_c = (int)std::max<int64_t>(1, std::min<int64_t>((capacity + 255) / 256, (int64_t)cus * 8));
  hipLaunchKernelGGL(k_cluster_clear, dim3(grid_t), dim3(256), 0, st, keys, t);
  hipLaunchKernelGGL(k_cluster_insert, dim3(grid_c), dim3(256), 0, st, c, count, capacity, keys, idx, log2t);
  hipLaunchKernelGGL(k_cluster_peaks, dim3(grid_c), dim3(256), 0, st, c, count, capacity, keys, idx, log2t, rr, rj,
                     keep);
  return hipGetLastError();
}

}  // namespace fdas
