// Host versions of the hipcub primitives the library calls, for the CPU
// emulation of its device code (hipemu.hpp).  Device-wide algorithms run as
// stream operations (recorded under graph capture); block-wide ones use the
// emulated block barrier, so every work-item of the block must call them.
#pragma once

#include <algorithm>
#include <numeric>
#include <vector>

#include "hipemu.hpp"

namespace hipcub {

namespace detail {
inline int flat_tid() {
  return (int)(threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z));
}
template <class K>
inline uint64_t key_bits(K k, int begin_bit, int end_bit) {
  uint64_t u = 0;
  std::memcpy(&u, &k, sizeof(K));
  if (std::is_signed<K>::value) u ^= 1ull << (8 * sizeof(K) - 1);  // order of signed keys
  if (sizeof(K) < 8) u &= (1ull << (8 * sizeof(K))) - 1;
  const int w = end_bit - begin_bit;
  u >>= begin_bit;
  if (w < 64) u &= (1ull << w) - 1;
  return u;
}
template <class K, class V>
void sort_pairs(const K* kin, K* kout, const V* vin, V* vout, int64_t n, int begin_bit, int end_bit) {
  std::vector<int64_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    return key_bits(kin[a], begin_bit, end_bit) < key_bits(kin[b], begin_bit, end_bit);
  });
  std::vector<K> ks(n);
  std::vector<V> vs(n);
  for (int64_t i = 0; i < n; ++i) {
    ks[i] = kin[idx[i]];
    vs[i] = vin[idx[i]];
  }
  for (int64_t i = 0; i < n; ++i) {
    kout[i] = ks[i];
    vout[i] = vs[i];
  }
}
}  // namespace detail

struct DeviceScan {
  template <class In, class Out>
  static hipError_t ExclusiveSum(void* tmp, size_t& bytes, In in, Out out, int n, hipStream_t s = nullptr,
                                 bool = false) {
    if (!tmp) {
      bytes = 256;
      return hipSuccess;
    }
    if (n < 0) return hipErrorInvalidValue;
    ::emu::stream_op(s, [in, out, n]() {
      using T = typename std::remove_reference<decltype(*out)>::type;
      T acc = 0;
      for (int i = 0; i < n; ++i) {
        const T v = (T)in[i];
        out[i] = acc;
        acc += v;
      }
    });
    return hipSuccess;
  }
};

struct DeviceRadixSort {
  template <class K, class V>
  static hipError_t SortPairs(void* tmp, size_t& bytes, const K* kin, K* kout, const V* vin, V* vout, int n,
                              int begin_bit = 0, int end_bit = sizeof(K) * 8, hipStream_t s = nullptr,
                              bool = false) {
    if (!tmp) {
      bytes = 256;
      return hipSuccess;
    }
    if (n < 0 || begin_bit < 0 || end_bit > (int)(8 * sizeof(K)) || begin_bit > end_bit) return hipErrorInvalidValue;
    ::emu::stream_op(s, [=]() { detail::sort_pairs(kin, kout, vin, vout, n, begin_bit, end_bit); });
    return hipSuccess;
  }
};

struct DeviceSegmentedRadixSort {
  template <class K, class V, class OffB, class OffE>
  static hipError_t SortPairs(void* tmp, size_t& bytes, const K* kin, K* kout, const V* vin, V* vout,
                              int num_items, int num_segments, OffB begin_off, OffE end_off, int begin_bit = 0,
                              int end_bit = sizeof(K) * 8, hipStream_t s = nullptr, bool = false) {
    if (!tmp) {
      bytes = 256;
      return hipSuccess;
    }
    if (num_items < 0 || num_segments < 0) return hipErrorInvalidValue;
    ::emu::stream_op(s, [=]() {
      for (int g = 0; g < num_segments; ++g) {
        const int64_t a = (int64_t)begin_off[g], b = (int64_t)end_off[g];
        if (a < 0 || b > num_items || a > b) ::emu::fail("segmented sort: segment %d [%lld, %lld) of %d items", g,
                                                         (long long)a, (long long)b, num_items);
        detail::sort_pairs(kin + a, kout + a, vin + a, vout + a, b - a, begin_bit, end_bit);
      }
    });
    return hipSuccess;
  }
};

template <class T, int BT, int ALG = 0, int BY = 1, int BZ = 1>
struct BlockScan {
  struct TempStorage {
    T v[BT * BY * BZ];
  };
  TempStorage& t;
  explicit BlockScan(TempStorage& s) : t(s) {}
  void ExclusiveSum(T in, T& out, T& total) {
    const int me = detail::flat_tid();
    t.v[me] = in;
    __syncthreads();
    T acc = 0, tot = 0;
    for (int i = 0; i < BT * BY * BZ; ++i) {
      if (i < me) acc += t.v[i];
      tot += t.v[i];
    }
    out = acc;
    total = tot;
    __syncthreads();
  }
  void ExclusiveSum(T in, T& out) {
    T tot;
    ExclusiveSum(in, out, tot);
  }
};

template <class K, int BT, int ITEMS, class V = int, int RADIX = 4, bool MEMOIZE = true, int ALG = 0,
          int BY = 1, int BZ = 1>
struct BlockRadixSort {
  struct TempStorage {
    K v[BT * BY * BZ * ITEMS];
  };
  TempStorage& t;
  explicit BlockRadixSort(TempStorage& s) : t(s) {}
  // blocked arrangement: work-item i holds sorted positions i*ITEMS ..
  void Sort(K (&keys)[ITEMS]) {
    const int me = detail::flat_tid();
    for (int i = 0; i < ITEMS; ++i) t.v[me * ITEMS + i] = keys[i];
    __syncthreads();
    if (me == 0) std::stable_sort(t.v, t.v + BT * BY * BZ * ITEMS);
    __syncthreads();
    for (int i = 0; i < ITEMS; ++i) keys[i] = t.v[me * ITEMS + i];
    __syncthreads();
  }
};

}  // namespace hipcub
