// Runtime of the CPU emulation of the HIP device model (see hipemu.hpp).
#include "hipemu.hpp"

#include <sanitizer/common_interface_defs.h>
#include <sys/mman.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <memory>
#include <mutex>
#include <thread>

// Context switch between fiber stacks (x86-64 System V): saves the
// callee-saved registers on the current stack, stores the stack pointer in
// *save, and resumes the stack `to` by popping its registers.  A new fiber's
// stack is laid out as if it had switched away just before its entry
// function (see Worker::prime).
extern "C" void emu_switch(void** save, void* to);
asm(R"(
  .text
  .globl emu_switch
  .type emu_switch, @function
emu_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
  .size emu_switch, .-emu_switch
)");

namespace emu {

thread_local Fiber* g_cur = nullptr;
thread_local BlockCtx g_blk;

struct Stream {
  bool capturing = false;
  Graph* graph = nullptr;
};
struct Event {
  std::chrono::steady_clock::time_point t;
};
struct Graph {
  std::vector<std::function<void()>> ops;
};

namespace {

constexpr size_t kStack = 512 * 1024;   // per work-item fiber (AddressSanitizer frames are large)
constexpr size_t kGuard = 4096;

std::mutex g_fail_mu;

struct Wave {
  int live = 0;
  int arrived = 0;
  int64_t seq = 0;           // completed collectives
  uint64_t arrived_mask = 0;
  uint64_t mask[2] = {0, 0};
  uint64_t slot[2][64];
  int kind = 0;
};

// One block in flight on a host thread.
struct SwCtx {
  void* sp = nullptr;
  const void* bottom = nullptr;   // lowest address of the stack (for the sanitizer)
  size_t size = 0;
  void* fake = nullptr;           // sanitizer fake-stack handle
};

struct BlockRun {
  std::vector<Fiber> fibers;
  std::vector<SwCtx> ctx;
  std::vector<Wave> waves;
  SwCtx sched;
  int nthreads = 0, live = 0;
  int bar_arrived = 0;
  int64_t bar_gen = 0;
  const std::function<void()>* body = nullptr;
};

thread_local BlockRun* t_run = nullptr;

struct Worker {
  std::vector<char*> stacks;
  BlockRun run;
  char* stack(size_t i) {
    while (stacks.size() <= i) {
      void* p = mmap(nullptr, kStack + kGuard, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE,
                     -1, 0);
      if (p == MAP_FAILED) fail("cannot map a fiber stack");
      mprotect(p, kGuard, PROT_NONE);   // overflow faults instead of corrupting the neighbour
      stacks.push_back(static_cast<char*>(p) + kGuard);
    }
    return stacks[i];
  }
};

void complete_wave(Wave& w) {
  w.mask[w.seq & 1] = w.arrived_mask;
  ++w.seq;
  w.arrived = 0;
  w.arrived_mask = 0;
  w.kind = 0;
}

void complete_barrier(BlockRun& r) {
  ++r.bar_gen;
  r.bar_arrived = 0;
}

// from -> to; returns when something switches back to `from`
void switch_ctx(SwCtx& from, SwCtx& to) {
  __sanitizer_start_switch_fiber(&from.fake, to.bottom, to.size);
  emu_switch(&from.sp, to.sp);
  __sanitizer_finish_switch_fiber(from.fake, nullptr, nullptr);
}

void yield_to_scheduler(Fiber* f) {
  BlockRun& r = *t_run;
  switch_ctx(r.ctx[f->flat], r.sched);
}

extern "C" void emu_fiber_entry() {
  BlockRun& r = *t_run;
  __sanitizer_finish_switch_fiber(nullptr, &r.sched.bottom, &r.sched.size);
  Fiber* f = g_cur;
  (*r.body)();
  f->done = true;
  Wave& w = r.waves[f->wave];
  --w.live;
  --r.live;
  if (w.arrived > 0 && w.arrived == w.live) complete_wave(w);
  if (r.bar_arrived > 0 && r.bar_arrived == r.live) complete_barrier(r);
  __sanitizer_start_switch_fiber(nullptr, r.sched.bottom, r.sched.size);   // this stack is finished
  void* dead;
  emu_switch(&dead, r.sched.sp);
  fail("finished work-item resumed");
}

void run_block(Worker& wk, const std::function<void()>& body, dim3 bid, dim3 bdim, dim3 gdim, const char* name) {
  BlockRun& r = wk.run;
  t_run = &r;
  g_blk.bid = bid;
  g_blk.bdim = bdim;
  g_blk.gdim = gdim;
  g_blk.kernel = name;
  const int nt = (int)(bdim.x * bdim.y * bdim.z);
  r.nthreads = nt;
  r.live = nt;
  r.bar_arrived = 0;
  r.bar_gen = 0;
  r.body = &body;
  r.fibers.assign(nt, Fiber());
  r.ctx.assign(nt, SwCtx());
  const int nw = (nt + 63) / 64;
  r.waves.assign(nw, Wave());
  for (int i = 0; i < nt; ++i) {
    Fiber& f = r.fibers[i];
    f.flat = i;
    f.tid = dim3(i % bdim.x, (i / bdim.x) % bdim.y, i / (bdim.x * bdim.y));
    f.lane = i & 63;
    f.wave = i >> 6;
    f.stack = wk.stack(i);
    SwCtx& c = r.ctx[i];
    c.bottom = f.stack;
    c.size = kStack;
    // entry frame: six zero registers, then emu_fiber_entry as the return
    // address of the switch, then a zero return address for the entry
    // function itself (keeps the ABI's 16-byte call alignment)
    uint64_t* top = reinterpret_cast<uint64_t*>(f.stack + kStack);
    top[-1] = 0;
    top[-2] = reinterpret_cast<uint64_t>(&emu_fiber_entry);
    for (int q = 3; q <= 8; ++q) top[-q] = 0;
    c.sp = top - 8;
    r.waves[f.wave].live++;
  }
  while (r.live > 0) {
    bool progress = false;
    for (int i = 0; i < nt; ++i) {
      Fiber& f = r.fibers[i];
      if (f.done) continue;
      if (f.wait == 1 && r.waves[f.wave].seq <= f.wait_val) continue;
      if (f.wait == 2 && r.bar_gen <= f.wait_val) continue;
      f.wait = 0;
      g_cur = &f;
      switch_ctx(r.sched, r.ctx[i]);
      progress = true;
    }
    if (!progress) {
      std::string who;
      for (int i = 0; i < nt && who.size() < 600; ++i) {
        const Fiber& f = r.fibers[i];
        if (f.done) continue;
        char b[96];
        std::snprintf(b, sizeof(b), " t%d:%s", i, f.wait == 1 ? "collective" : (f.wait == 2 ? "barrier" : "?"));
        who += b;
      }
      fail("deadlock in block (%u,%u,%u):%s", bid.x, bid.y, bid.z, who.c_str());
    }
  }
  g_cur = nullptr;
  t_run = nullptr;
}

// Host-thread pool running the blocks of one launch at a time.
struct Pool {
  std::vector<std::thread> threads;
  std::vector<std::unique_ptr<Worker>> workers;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  uint64_t job = 0;
  int running = 0;
  const std::function<void()>* body = nullptr;
  dim3 grid, block;
  const char* name = "";
  std::atomic<int64_t> next{0};
  int64_t total = 0;
  bool stop = false;

  explicit Pool(int n) {
    for (int i = 0; i < n; ++i) workers.emplace_back(new Worker());
    for (int i = 1; i < n; ++i) threads.emplace_back([this, i] { loop(i); });
  }
  void work(int i) {
    for (;;) {
      const int64_t b = next.fetch_add(1);
      if (b >= total) break;
      const dim3 bid((unsigned)(b % grid.x), (unsigned)((b / grid.x) % grid.y), (unsigned)(b / ((int64_t)grid.x * grid.y)));
      run_block(*workers[i], *body, bid, block, grid, name);
    }
  }
  void loop(int i) {
    uint64_t seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> l(mu);
        cv.wait(l, [&] { return stop || job != seen; });
        if (stop) return;
        seen = job;
      }
      work(i);
      {
        std::lock_guard<std::mutex> l(mu);
        if (--running == 0) done_cv.notify_all();
      }
    }
  }
  void launch(const std::function<void()>& b, dim3 g, dim3 bl, const char* nm) {
    {
      std::lock_guard<std::mutex> l(mu);
      body = &b;
      grid = g;
      block = bl;
      name = nm;
      total = (int64_t)g.x * g.y * g.z;
      next = 0;
      running = (int)threads.size();
      ++job;
    }
    cv.notify_all();
    work(0);
    std::unique_lock<std::mutex> l(mu);
    done_cv.wait(l, [&] { return running == 0; });
  }
};

Pool& pool() {
  static Pool* p = [] {
    int n = 8;
    if (const char* e = std::getenv("EMU_THREADS")) n = std::max(1, std::atoi(e));
    return new Pool(n);
  }();
  return *p;
}

std::mutex g_launch_mu;
hipError_t g_last = hipSuccess;
std::atomic<int64_t> g_launches{0};

}  // namespace

void fail(const char* fmt, ...) {
  std::lock_guard<std::mutex> l(g_fail_mu);
  std::fprintf(stderr, "\n[hipemu] ");
  if (g_cur)
    std::fprintf(stderr, "kernel %s block (%u,%u,%u) thread (%u,%u,%u): ", g_blk.kernel, g_blk.bid.x, g_blk.bid.y,
                 g_blk.bid.z, g_cur->tid.x, g_cur->tid.y, g_cur->tid.z);
  va_list ap;
  va_start(ap, fmt);
  std::vfprintf(stderr, fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "\n");
  std::fflush(stderr);
  std::abort();
}

const uint64_t* wave_collect(uint64_t v, uint64_t* mask, int kind) {
  Fiber* f = g_cur;
  if (!f) fail("wavefront collective outside a kernel");
  BlockRun& r = *t_run;
  Wave& w = r.waves[f->wave];
  const int64_t k = w.seq;
  if (w.arrived == 0) {
    w.kind = kind;
  } else if (w.kind != kind) {
    fail("divergent wavefront collective: lanes of wave %d wait at collectives of kinds %d and %d", f->wave,
         w.kind, kind);
  }
  w.slot[k & 1][f->lane] = v;
  ++w.arrived;
  w.arrived_mask |= 1ull << f->lane;
  if (w.arrived == w.live) {
    complete_wave(w);
  } else {
    f->wait = 1;
    f->wait_val = k;
    yield_to_scheduler(f);
  }
  *mask = w.mask[k & 1];
  return w.slot[k & 1];
}

void block_barrier() {
  Fiber* f = g_cur;
  if (!f) fail("__syncthreads outside a kernel");
  BlockRun& r = *t_run;
  if (r.waves[f->wave].arrived > 0) fail("__syncthreads while lanes of the same wavefront wait at a collective");
  const int64_t gen = r.bar_gen;
  ++r.bar_arrived;
  if (r.bar_arrived == r.live) {
    complete_barrier(r);
  } else {
    f->wait = 2;
    f->wait_val = gen;
    yield_to_scheduler(f);
  }
}

void stream_op(hipStream_t s, std::function<void()> op) {
  if (s && s->capturing) {
    s->graph->ops.push_back(std::move(op));
    return;
  }
  op();
}

void submit_launch(const char* name, dim3 grid, dim3 block, hipStream_t s, std::function<void()> body) {
  const int64_t nt = (int64_t)block.x * block.y * block.z;
  if (nt < 1 || nt > 1024 || grid.x < 1 || grid.y < 1 || grid.z < 1 || grid.x > 0x7fffffffu || grid.y > 65535 ||
      grid.z > 65535) {
    std::fprintf(stderr, "[hipemu] launch of %s with grid (%u,%u,%u) block (%u,%u,%u) is invalid\n", name, grid.x,
                 grid.y, grid.z, block.x, block.y, block.z);
    g_last = hipErrorInvalidConfiguration;
    return;
  }
  auto run = [name, grid, block, body]() {
    std::lock_guard<std::mutex> l(g_launch_mu);
    const auto t0 = std::chrono::steady_clock::now();
    pool().launch(body, grid, block, name);
    ++g_launches;
    if (std::getenv("EMU_TRACE"))
      std::fprintf(stderr, "[hipemu] %s grid (%u,%u,%u) block (%u,%u,%u) %.1f ms\n", name, grid.x, grid.y, grid.z,
                   block.x, block.y, block.z,
                   std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
  };
  stream_op(s, run);
}

}  // namespace emu

using emu::Event;
using emu::Graph;
using emu::Stream;

hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidValue; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  std::memset(p, 0, sizeof(*p));
  std::snprintf(p->name, sizeof(p->name), "host emulation");
  std::snprintf(p->gcnArchName, sizeof(p->gcnArchName), "emu-gfx950:sramecc+:xnack-");
  p->totalGlobalMem = (size_t)288 << 30;
  p->sharedMemPerBlock = 160 * 1024;
  p->multiProcessorCount = 256;
  p->warpSize = 64;
  p->maxThreadsPerBlock = 1024;
  return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t bytes) {
  void* q = nullptr;
  if (posix_memalign(&q, 256, bytes ? bytes : 1) != 0) return hipErrorOutOfMemory;
  // device memory starts with arbitrary contents: make that visible
  std::memset(q, 0xA5, bytes);
  *p = q;
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemGetInfo(size_t* free_b, size_t* total_b) {
  *free_b = (size_t)64 << 30;
  *total_b = (size_t)288 << 30;
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  if (bytes) std::memmove(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  emu::stream_op(s, [=] {
    if (bytes) std::memmove(dst, src, bytes);
  });
  return hipSuccess;
}
hipError_t hipMemset(void* dst, int v, size_t bytes) {
  if (bytes) std::memset(dst, v, bytes);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t s) {
  emu::stream_op(s, [=] {
    if (bytes) std::memset(dst, v, bytes);
  });
  return hipSuccess;
}
hipError_t hipStreamCreate(hipStream_t* s) {
  *s = new Stream();
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { return hipStreamCreate(s); }
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  if (s && s->capturing) return hipErrorInvalidValue;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (!s || s->capturing) return hipErrorInvalidValue;
  s->capturing = true;
  s->graph = new Graph();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  if (!s || !s->capturing) return hipErrorInvalidValue;
  s->capturing = false;
  *g = s->graph;
  s->graph = nullptr;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *e = new Graph(*g);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s) {
  if (s && s->capturing) return hipErrorInvalidValue;
  for (auto& op : e->ops) op();
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = new Event();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  emu::stream_op(s, [e] { e->t = std::chrono::steady_clock::now(); });
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() {
  const hipError_t e = emu::g_last;
  emu::g_last = hipSuccess;
  return e;
}
const char* hipGetErrorString(hipError_t e) {
  switch (e) {
    case hipSuccess: return "hipSuccess";
    case hipErrorInvalidValue: return "hipErrorInvalidValue";
    case hipErrorOutOfMemory: return "hipErrorOutOfMemory";
    case hipErrorInvalidConfiguration: return "hipErrorInvalidConfiguration";
    default: return "hipError (emulated)";
  }
}
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
