// CPU emulation of the HIP device model, for running the library's own
// kernel sources on the host under AddressSanitizer (test infrastructure:
// it checks every global-memory access of the device code against the
// exact allocation it belongs to, which a GPU cannot do).
//
// Execution model: a launch runs its blocks on a pool of host threads; in
// each block every work-item is a fiber with its own stack and the fibers of a
// block are scheduled cooperatively on one host thread (a register-saving
// stack switch, announced to the sanitizer as a fiber switch).  A work-item runs
// until it reaches a synchronisation point:
//   * a wavefront collective (DPP row broadcast, shuffle, ballot, any,
//     readlane, the FP64 matrix-core product, wave barrier): every live
//     lane of the 64-lane wavefront must arrive at a collective of the same
//     kind, and
//     then all of them see all lanes' operands, as in lockstep execution;
//   * __syncthreads(): every live work-item of the block must arrive.
// Lanes that have returned take no part (they are the lanes a hardware
// wavefront has switched off for good).  A wavefront whose live lanes wait
// at collectives of different kinds, or a block whose work-items cannot all make
// progress, stops the run with a report (divergent collective / deadlock).
// LDS (__shared__) is a thread_local static: one copy per host thread, so
// per running block.  Streams are synchronous; graph capture records
// launches and copies, and a graph launch replays them.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <tuple>
#include <type_traits>
#include <utility>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __constant__
#define __shared__ static thread_local
#define __forceinline__ inline
#define __noinline__ __attribute__((noinline))
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
#define __restrict__ __restrict

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

struct __attribute__((aligned(8))) int2 { int x, y; };
struct __attribute__((aligned(16))) int4 { int x, y, z, w; };
struct __attribute__((aligned(16))) double2 { double x, y; };
struct __attribute__((aligned(32))) double4 { double x, y, z, w; };
inline int2 make_int2(int x, int y) { return int2{x, y}; }
inline int4 make_int4(int x, int y, int z, int w) { return int4{x, y, z, w}; }
inline double2 make_double2(double x, double y) { return double2{x, y}; }
inline double4 make_double4(double x, double y, double z, double w) { return double4{x, y, z, w}; }

// ---------------------------------------------------------------- runtime
enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidConfiguration = 9,
  hipErrorLaunchFailure = 719,
  hipErrorUnknown = 999,
};
enum hipMemcpyKind {
  hipMemcpyHostToHost = 0,
  hipMemcpyHostToDevice = 1,
  hipMemcpyDeviceToHost = 2,
  hipMemcpyDeviceToDevice = 3,
  hipMemcpyDefault = 4,
};
enum hipStreamCaptureMode {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal = 1,
  hipStreamCaptureModeRelaxed = 2,
};
#define hipStreamNonBlocking 1u

namespace emu {
struct Stream;
struct Event;
struct Graph;
}  // namespace emu
typedef emu::Stream* hipStream_t;
typedef emu::Event* hipEvent_t;
typedef emu::Graph* hipGraph_t;
typedef emu::Graph* hipGraphExec_t;
typedef void* hipGraphNode_t;

struct hipDeviceProp_t {
  char name[256];
  char gcnArchName[256];
  size_t totalGlobalMem;
  size_t sharedMemPerBlock;
  int multiProcessorCount;
  int warpSize;
  int maxThreadsPerBlock;
  int clockRate;
  int l2CacheSize;
};

hipError_t hipGetDeviceCount(int* n);
hipError_t hipSetDevice(int d);
hipError_t hipGetDevice(int* d);
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int d);
hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipMemGetInfo(size_t* free_b, size_t* total_b);
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind k, hipStream_t s = nullptr);
hipError_t hipMemset(void* dst, int v, size_t bytes);
hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t s = nullptr);
hipError_t hipStreamCreate(hipStream_t* s);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t* err_node, char* log, size_t n);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipGetSymbolAddress(void** p, const void* symbol);
#define HIP_SYMBOL(x) ((const void*)&(x))

// Blocks per CU of a kernel: the emulator has no occupancy model; 3 is what
// the update kernels reach on gfx950 (3 waves per SIMD, 4 waves per block).
template <class F>
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* nb, F, int, size_t) {
  *nb = 3;
  return hipSuccess;
}

namespace emu {

struct Fiber {
  dim3 tid;
  int flat = 0, lane = 0, wave = 0;
  char* stack = nullptr;
  bool done = false;
  int wait = 0;             // 0 none, 1 wave collective, 2 block barrier
  int64_t wait_val = 0;
};

struct BlockCtx {
  dim3 bid, bdim, gdim;
  const char* kernel = "";
};

extern thread_local Fiber* g_cur;
extern thread_local BlockCtx g_blk;

[[noreturn]] void fail(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

// Kinds of wavefront collectives.  Lanes of one wavefront must meet at
// collectives of the same kind (a host compiler may duplicate code, so the
// call site itself is not a usable identity).
enum Kind { kDpp = 1, kReadlane, kWaveBarrier, kMfmaA, kMfmaB, kShfl, kVote };

// Wavefront collective: deposits v for the calling lane, waits until every
// live lane of the wavefront has arrived at a collective of the same kind,
// and returns the 64 deposited values; *mask receives the lanes that took
// part.
const uint64_t* wave_collect(uint64_t v, uint64_t* mask, int kind);
void block_barrier();

// Work of a launch (run per work-item) and of host-side stream operations.
void submit_launch(const char* name, dim3 grid, dim3 block, hipStream_t s, std::function<void()> body);
void stream_op(hipStream_t s, std::function<void()> op);

struct Cfg {
  dim3 grid, block;
  hipStream_t stream;
  Cfg(dim3 g, dim3 b, size_t = 0, hipStream_t s = nullptr) : grid(g), block(b), stream(s) {}
  template <class F, class... A>
  void launch(const char* name, F f, A&&... a) {
    auto args = std::make_tuple(std::decay_t<A>(std::forward<A>(a))...);
    submit_launch(name, grid, block, stream, [f, args]() { std::apply(f, args); });
  }
};

template <class T>
inline uint64_t to_bits(T v) {
  static_assert(sizeof(T) <= 8, "collective operand wider than 64 bits");
  uint64_t b = 0;
  std::memcpy(&b, &v, sizeof(T));
  return b;
}
template <class T>
inline T from_bits(uint64_t b) {
  T v;
  std::memcpy(&v, &b, sizeof(T));
  return v;
}

inline int lane() { return g_cur->lane; }

// DPP row_newbcast:u (control 0x150 + u): every lane of a 16-lane row gets
// lane u of its row; a source lane that is not live leaves `old`.
inline int update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
  if (ctrl < 0x150 || ctrl > 0x15F || row_mask != 0xF || bank_mask != 0xF || bound_ctrl)
    fail("update_dpp: control 0x%x (row_mask %x bank_mask %x bound_ctrl %d) is not emulated", ctrl, row_mask,
         bank_mask, (int)bound_ctrl);
  uint64_t m;
  const uint64_t* all = wave_collect(to_bits((uint32_t)src), &m, kDpp);
  const int s = (lane() & ~15) + (ctrl - 0x150);
  return (m >> s & 1) ? (int)(uint32_t)all[s] : old;
}

inline int readlane(int v, int l) {
  uint64_t m;
  const uint64_t* all = wave_collect(to_bits((uint32_t)v), &m, kReadlane);
  if (l < 0 || l > 63 || !(m >> l & 1)) fail("readlane of lane %d, which is not live", l);
  return (int)(uint32_t)all[l];
}

// v_readfirstlane: the value of the lowest live lane, in every lane.
inline int readfirstlane(int v) {
  uint64_t m;
  const uint64_t* all = wave_collect(to_bits((uint32_t)v), &m, kReadlane);
  if (!m) fail("readfirstlane with no live lane");
  return (int)(uint32_t)all[__builtin_ctzll(m)];
}

inline uint32_t mbcnt_lo(uint32_t mask, uint32_t acc) {
  const int l = lane();
  const uint32_t below = l >= 32 ? 0xffffffffu : ((1u << l) - 1u);
  return acc + (uint32_t)__builtin_popcount(mask & below);
}
inline uint32_t mbcnt_hi(uint32_t mask, uint32_t acc) {
  const int l = lane();
  const uint32_t below = l < 32 ? 0u : (l == 32 ? 0u : ((1u << (l - 32)) - 1u));
  return acc + (uint32_t)__builtin_popcount(mask & below);
}

inline void wave_barrier() {
  uint64_t m;
  (void)wave_collect(0, &m, kWaveBarrier);
}

typedef double d4v __attribute__((ext_vector_type(4)));
// v_mfma_f64_16x16x4f64: D[16x16] = A[16x4] B[4x16] + C with lane l holding
// A[l % 16][l / 16], B[l / 16][l % 16] and D[4 v + l / 16][l % 16] in its
// v-th accumulator register.
inline d4v mfma_f64_16x16x4(double a, double b, d4v c, int cbsz, int abid, int blgp) {
  if (cbsz || abid || blgp) fail("mfma_f64_16x16x4f64 with broadcast controls is not emulated");
  uint64_t ma, mb;
  const uint64_t* A = wave_collect(to_bits(a), &ma, kMfmaA);
  double av[64];
  for (int i = 0; i < 64; ++i) av[i] = from_bits<double>(A[i]);
  const uint64_t* Bv = wave_collect(to_bits(b), &mb, kMfmaB);
  if (ma != ~0ull || mb != ~0ull) fail("matrix-core product with lanes that are not live (mask %llx)",
                                       (unsigned long long)ma);
  const int l = lane(), j = l & 15, g = l >> 4;
  d4v d = c;
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * v + g;
    double s = d[v];
    for (int k = 0; k < 4; ++k) s += av[k * 16 + i] * from_bits<double>(Bv[k * 16 + j]);
    d[v] = s;
  }
  return d;
}

}  // namespace emu

#define threadIdx (::emu::g_cur->tid)
#define blockIdx (::emu::g_blk.bid)
#define blockDim (::emu::g_blk.bdim)
#define gridDim (::emu::g_blk.gdim)

#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) ::emu::update_dpp((old), (src), (ctrl), (rm), (bm), (bc))
#define __builtin_amdgcn_readlane(v, l) ::emu::readlane((v), (l))
#define __builtin_amdgcn_readfirstlane(v) ::emu::readfirstlane((v))
#define __builtin_amdgcn_mbcnt_lo(m, a) ::emu::mbcnt_lo((m), (a))
#define __builtin_amdgcn_mbcnt_hi(m, a) ::emu::mbcnt_hi((m), (a))
#define __builtin_amdgcn_wave_barrier() ::emu::wave_barrier()
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) ::emu::mfma_f64_16x16x4((a), (b), (c), (x), (y), (z))

inline void __syncthreads() { ::emu::block_barrier(); }

template <class T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  uint64_t m;
  const uint64_t* all = ::emu::wave_collect(::emu::to_bits(v), &m, ::emu::kShfl);
  const int l = ::emu::lane();
  const int src = (l & ~(width - 1)) | ((l ^ mask) & (width - 1));
  if (!(m >> src & 1)) ::emu::fail("__shfl_xor from lane %d, which is not live", src);
  return ::emu::from_bits<T>(all[src]);
}

template <class T>
inline T __shfl_up(T v, unsigned delta, int width = 64) {
  uint64_t m;
  const uint64_t* all = ::emu::wave_collect(::emu::to_bits(v), &m, ::emu::kShfl);
  const int l = ::emu::lane();
  if ((l & (width - 1)) < (int)delta) return v;
  const int src = l - (int)delta;
  if (!(m >> src & 1)) ::emu::fail("__shfl_up from lane %d, which is not live", src);
  return ::emu::from_bits<T>(all[src]);
}

inline int __any(int p) {
  uint64_t m;
  const uint64_t* all = ::emu::wave_collect(p ? 1 : 0, &m, ::emu::kVote);
  for (int i = 0; i < 64; ++i)
    if ((m >> i & 1) && all[i]) return 1;
  return 0;
}
inline int __all(int p) {
  uint64_t m;
  const uint64_t* all = ::emu::wave_collect(p ? 1 : 0, &m, ::emu::kVote);
  for (int i = 0; i < 64; ++i)
    if ((m >> i & 1) && !all[i]) return 0;
  return 1;
}
inline unsigned long long __ballot(int p) {
  uint64_t m;
  const uint64_t* all = ::emu::wave_collect(p ? 1 : 0, &m, ::emu::kVote);
  unsigned long long r = 0;
  for (int i = 0; i < 64; ++i)
    if ((m >> i & 1) && all[i]) r |= 1ull << i;
  return r;
}

#define __HIP_MEMORY_SCOPE_WAVEFRONT 2
#define __HIP_MEMORY_SCOPE_WORKGROUP 3
#define __HIP_MEMORY_SCOPE_AGENT 4
#define __HIP_MEMORY_SCOPE_SYSTEM 5
#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), (order))
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n((p), (v), (order))
#define __builtin_amdgcn_s_sleep(n) ((void)0)

inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __popc(unsigned v) { return __builtin_popcount(v); }
inline long long __double_as_longlong(double v) { return ::emu::from_bits<long long>(::emu::to_bits(v)); }
inline double __longlong_as_double(long long v) { return ::emu::from_bits<double>(::emu::to_bits(v)); }

template <class T>
inline T atomicAdd(T* p, T v) {
  return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
inline double atomicAdd(double* p, double v) {
  uint64_t* q = reinterpret_cast<uint64_t*>(p);
  uint64_t ob = __atomic_load_n(q, __ATOMIC_SEQ_CST);
  for (;;) {
    const uint64_t nb = ::emu::to_bits(::emu::from_bits<double>(ob) + v);
    if (__atomic_compare_exchange_n(q, &ob, nb, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST))
      return ::emu::from_bits<double>(ob);
  }
}
template <class T>
inline T atomicOr(T* p, T v) {
  return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST);
}
template <class T>
inline T atomicMax(T* p, T v) {
  T cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (cur < v && !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
  }
  return cur;
}

using std::isfinite;
using std::isinf;
using std::isnan;

// device-side min / max overloads of HIP
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
inline unsigned max(unsigned a, unsigned b) { return a > b ? a : b; }
inline long min(long a, long b) { return a < b ? a : b; }
inline long max(long a, long b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
inline long long max(long long a, long long b) { return a > b ? a : b; }
inline unsigned long min(unsigned long a, unsigned long b) { return a < b ? a : b; }
inline unsigned long max(unsigned long a, unsigned long b) { return a > b ? a : b; }
inline unsigned long long min(unsigned long long a, unsigned long long b) { return a < b ? a : b; }
inline unsigned long long max(unsigned long long a, unsigned long long b) { return a > b ? a : b; }
inline double min(double a, double b) { return fmin(a, b); }
inline double max(double a, double b) { return fmax(a, b); }
inline float min(float a, float b) { return fminf(a, b); }
inline float max(float a, float b) { return fmaxf(a, b); }
