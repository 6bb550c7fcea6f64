// Batched gamma_2: many (n, m) instances in one persistent launch.
//
// gamma_2(P_n x C_m) = min_i (A^m)_ii (Theorem 2) = trace of A^a x A^b for any
// a + b = m.  A context keeps, per path order n, the powers A^1 .. A^K of the
// chain A^k = A x A^(k-1) (Algorithm 2) resident in HBM; every instance with
// that n reads its answer from two of them (a = ceil(m/2), b = floor(m/2))
// with one trace of a product.  A batch therefore costs one chain per
// distinct n (only the levels not already resident) plus one trace per
// instance.
//
// The work of a batch is a queue of tasks in dependency order:
//   BUILD  rows of A^1 = A(D_n)
//   SPMM   rows of A^k = A x A^(k-1) (needs all of level k-1 of that n)
//   TRACE  64 rows i of min_{i,k} (A^a)_ik + (A^b)_ki for one instance
//          (needs level a of that n), folded into the instance's result
// A persistent kernel pops tasks in queue order with an atomic counter.  A
// task waits only for tasks that precede it in the queue, which were popped
// earlier by running workgroups, so the wait always ends; as a safety net
// every wait is bounded in time, and a timed-out wait sets an abort flag that
// makes every workgroup drain the queue without work.  Finished tasks publish
// their rows with an agent-scope release (so other XCDs' L2s see them) and a
// counter increment; waiting tasks acquire before reading.  Levels of
// different n interleave in the queue, so small and large chains overlap on
// the device.  The launch (counter reset, result reset, persistent kernel) is
// captured once in a hipGraph and replayed for every batch.
#include <stdarg.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "device_core.hpp"

namespace tp {

namespace {

enum : int32_t { kBuild = 0, kSpmm = 1, kTrace = 2 };

struct Task {
  int32_t type, slot;
  int32_t a, b;        // level written (BUILD, SPMM) or the two powers (TRACE)
  int32_t row0, row1;  // output rows, or the 64 rows i of a trace
  int32_t dep, dep_target;  // counter to wait for (-1: none) and the count it must reach
  int32_t done;             // counter bumped when finished (-1: none)
  int32_t inst;             // instance of a TRACE
};

struct Slot {
  int32_t n, N;
  int64_t ld;
  uint32_t full;
  int32_t pad;
  const uint32_t *masks;
  const int64_t *rowptr;
  const uint32_t *col;
  const uint8_t *z;
  uint16_t *const *powers;  // powers[k - 1] = A^k
};

struct Control {
  int32_t head;      // next task to pop
  int32_t ntasks;
  int32_t abort;     // set when a wait exceeded the limit
  int32_t pad;
  int64_t wait_limit;  // in s_memrealtime ticks (100 MHz)
};

constexpr int kMaxSlots = 16;
constexpr uint16_t kInf = 0xFFFFu;

__device__ __forceinline__ int32_t ld_relaxed(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(256) batch_kernel(Control *__restrict__ ctl,
                                                    const Task *__restrict__ tasks,
                                                    const Slot *__restrict__ slots,
                                                    int32_t *__restrict__ counters,
                                                    int32_t *__restrict__ results) {
  __shared__ __attribute__((aligned(16))) uint16_t yt[64 * kTraceLdsStride];
  __shared__ int32_t part[4];
  __shared__ int32_t s_task, s_go;
  const int ntasks = ctl->ntasks;
  const int64_t limit = ctl->wait_limit;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  while (true) {
    if (threadIdx.x == 0) {
      const int t = atomicAdd(&ctl->head, 1);
      int go = 0;
      if (t < ntasks) {
        go = ld_relaxed(&ctl->abort) == 0;
        const int dep = tasks[t].dep;
        if (go && dep >= 0) {
          const int target = tasks[t].dep_target;
          const uint64_t start = __builtin_amdgcn_s_memrealtime();
          while (ld_relaxed(&counters[dep]) < target) {
            if (ld_relaxed(&ctl->abort)) {
              go = 0;
              break;
            }
            if ((int64_t)(__builtin_amdgcn_s_memrealtime() - start) > limit) {
              __hip_atomic_store(&ctl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              go = 0;
              break;
            }
            __builtin_amdgcn_s_sleep(2);
          }
        }
      }
      s_task = t;
      s_go = go;
    }
    __syncthreads();
    const int t = s_task;
    const int go = s_go;
    if (t >= ntasks) break;
    const Task task = tasks[t];
    if (go) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const Slot sl = slots[task.slot];
      const int64_t N = sl.N, ld = sl.ld;
      if (task.type == kBuild) {
        uint16_t *out = sl.powers[0];
        const int64_t rows = task.row1 - task.row0;
        for (int64_t idx = threadIdx.x; idx < rows * N; idx += blockDim.x) {
          const int64_t q = task.row0 + idx / N, p = idx - (idx / N) * N;
          const uint32_t mp = sl.masks[p];
          out[q * ld + p] = can_follow(sl.masks[q], mp, sl.full)
                                ? (uint16_t)__builtin_popcount(mp & 0xFFFFu)
                                : kInf;
        }
      } else if (task.type == kSpmm) {
        const uint16_t *X = sl.powers[task.a - 2];
        uint16_t *Y = sl.powers[task.a - 1];
        for (int64_t q = task.row0 + wave; q < task.row1; q += 4) {
          const int64_t qu = __builtin_amdgcn_readfirstlane((int)q);
          for (int64_t c0 = (int64_t)lane * 8; c0 < N; c0 += 512)
            spmm_row_chunk<uint16_t, true>(sl.rowptr, sl.col, sl.z, X, ld, Y, ld, N, qu, c0);
        }
      } else {
        const uint16_t *X = sl.powers[task.a - 1];
        const uint16_t *Y = sl.powers[task.b - 1];
        u16x2 acc[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = splat(kInf);
        for (int64_t k0 = 0; k0 < N; k0 += 64)
          trace_tile<uint16_t, true>(X, ld, Y, ld, N, task.row0, k0, yt, acc);
        const int32_t best = block_min(acc, part);
        if (threadIdx.x == 0 && best < (int32_t)kInf) atomicMin(&results[task.inst], best);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    __syncthreads();
    if (threadIdx.x == 0 && task.done >= 0)
      __hip_atomic_fetch_add(&counters[task.done], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void fill_kernel(int32_t *p, int64_t count, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
};

hipError_t grow(Buf &b, size_t bytes) {
  if (b.p && b.bytes >= bytes) return hipSuccess;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    if (e != hipSuccess) return e;
  }
  b.p = nullptr;
  b.bytes = 0;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e == hipSuccess) b.bytes = bytes;
  return e;
}

hipError_t grow_host(Buf &b, size_t bytes) {
  if (b.p && b.bytes >= bytes) return hipSuccess;
  if (b.p) {
    hipError_t e = hipHostFree(b.p);
    if (e != hipSuccess) return e;
  }
  b.p = nullptr;
  b.bytes = 0;
  hipError_t e = hipHostMalloc(&b.p, bytes, hipHostMallocDefault);
  if (e == hipSuccess) b.bytes = bytes;
  return e;
}

struct PowerSet {
  int64_t N = 0, ld = 0;
  std::vector<void *> pw;  // pw[k - 1] = A^k
  int have = 0;            // powers known complete on the device
};

}  // namespace

struct Ctx {
  int device = 0;
  size_t budget = 0, used = 0;
  std::map<int, PowerSet> sets;
  Buf d_tasks, d_slots, d_ptrs, d_counters, d_results, d_ctl;
  Buf h_tasks, h_slots, h_ptrs, h_ctl, h_flag;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  void *g_key[3] = {nullptr, nullptr, nullptr};
  size_t g_counter_cap = 0, g_result_cap = 0;
  int g_grid = 0;
  hipEvent_t staged = nullptr;
  int64_t wait_limit = 2000000000;  // 20 s at 100 MHz
  int spmm_rows[16] = {0};          // rows per SPMM task by n; 0 = automatic
  int grid_override = 0;
  bool pending = false;  // a batch was queued and not yet checked
  std::vector<int> pending_n;
  std::vector<int> pending_have;
  std::mutex mu;
};

namespace {

int auto_spmm_rows(int64_t N, int64_t nnz) {
  // about 2^22 (min,+) operations per task, a multiple of 4 rows (one per wave)
  const double per_row = (double)nnz / (double)N * (double)N;
  int64_t r = (int64_t)(4194304.0 / std::max(per_row, 1.0));
  r = std::max<int64_t>(4, std::min<int64_t>(r, 256));
  return (int)((r + 3) / 4 * 4);
}

int capture_graph(Ctx *c, int grid) {
  if (c->exec) {
    (void)hipGraphExecDestroy(c->exec);
    c->exec = nullptr;
  }
  if (!c->cap_stream) TP_HIP_CHECK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  TP_HIP_CHECK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
  const int64_t nc = (int64_t)(c->d_counters.bytes / sizeof(int32_t));
  const int64_t nr = (int64_t)(c->d_results.bytes / sizeof(int32_t));
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, c->cap_stream,
                     (int32_t *)c->d_counters.p, nc, 0);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, c->cap_stream,
                     (int32_t *)c->d_results.p, nr, (int32_t)kInf);
  hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(256), 0, c->cap_stream, (Control *)c->d_ctl.p,
                     (const Task *)c->d_tasks.p, (const Slot *)c->d_slots.p,
                     (int32_t *)c->d_counters.p, (int32_t *)c->d_results.p);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&c->exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  c->g_key[0] = c->d_tasks.p;
  c->g_key[1] = c->d_counters.p;
  c->g_key[2] = c->d_results.p;
  c->g_counter_cap = c->d_counters.bytes;
  c->g_result_cap = c->d_results.bytes;
  c->g_grid = grid;
  return TP_OK;
}

int default_grid() {
  int dev = 0, cus = 0, per_cu = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel, 256, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 4;
  return cus * per_cu;
}

}  // namespace

int batch_run(Ctx *c, int count, const int32_t *ns, const int64_t *ms, int32_t *gamma2_dev,
              hipStream_t stream) {
  // wait until the previous batch's staging buffers have been consumed
  if (c->staged) TP_HIP_CHECK(hipEventSynchronize(c->staged));
  // distinct n, in increasing order, with the highest level each one needs
  std::map<int, int> need;  // n -> K = max ceil(m / 2)
  for (int j = 0; j < count; ++j) {
    const int a = (int)((ms[j] + 1) / 2);
    int &k = need[ns[j]];
    k = std::max(k, a);
  }
  TP_REQUIRE((int)need.size() <= kMaxSlots, "more than %d distinct n in one batch", kMaxSlots);
  std::map<int, int> slot_of;
  std::vector<StateView> views;
  int kmax = 0;
  for (auto &kv : need) {
    StateView v{};
    const int rc = state_view(kv.first, stream, &v);
    if (rc != TP_OK) return rc;
    slot_of[kv.first] = (int)views.size();
    views.push_back(v);
    kmax = std::max(kmax, kv.second);
    PowerSet &ps = c->sets[kv.first];
    ps.N = v.N;
    ps.ld = (v.N + 63) / 64 * 64;
    const size_t bytes = (size_t)ps.N * (size_t)ps.ld * sizeof(uint16_t);
    while ((int)ps.pw.size() < kv.second) {
      if (c->used + bytes > c->budget) {
        set_error("batch needs %d resident powers of A(D_%d) (%zu bytes each): over the budget of %zu bytes",
                  kv.second, kv.first, bytes, c->budget);
        return TP_ENOMEM;
      }
      void *p = nullptr;
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) return hip_fail(e, "hipMalloc (resident power)");
      c->used += bytes;
      ps.pw.push_back(p);
    }
  }
  const int nslots = (int)views.size();
  auto counter = [&](int slot, int level) { return slot * (kmax + 1) + level; };

  // tasks in dependency order: level by level over all n, traces right after
  // the level they read
  std::vector<Task> tasks;
  std::vector<std::vector<int>> level_tasks(nslots, std::vector<int>(kmax + 1, 0));
  std::vector<std::vector<int>> by_level(kmax + 1);
  for (int j = 0; j < count; ++j) by_level[(ms[j] + 1) / 2].push_back(j);
  auto push_traces = [&](int j) {
    const int s = slot_of[ns[j]];
    const PowerSet &ps = c->sets[ns[j]];
    const int a = (int)((ms[j] + 1) / 2), b = (int)(ms[j] / 2);
    const bool computed = a > ps.have;
    for (int64_t i0 = 0; i0 < ps.N; i0 += 64) {
      Task t{};
      t.type = kTrace;
      t.slot = s;
      t.a = a;
      t.b = b;
      t.row0 = (int32_t)i0;
      t.row1 = (int32_t)std::min<int64_t>(i0 + 64, ps.N);
      t.dep = computed ? counter(s, a) : -1;
      t.dep_target = computed ? level_tasks[s][a] : 0;
      t.done = -1;
      t.inst = j;
      tasks.push_back(t);
    }
  };
  for (int k = 1; k <= kmax; ++k) {
    for (int s = 0; s < nslots; ++s) {
      const int n = views[s].n;
      const PowerSet &ps = c->sets[n];
      if (k > need[n] || k <= ps.have) continue;
      const int64_t N = ps.N;
      int rows;
      if (k == 1)
        rows = (int)std::max<int64_t>(1, std::min<int64_t>(N, 262144 / std::max<int64_t>(N, 1)));
      else
        rows = c->spmm_rows[n] > 0 ? c->spmm_rows[n] : auto_spmm_rows(N, views[s].nnz);
      const bool dep = k >= 2 && (k - 1) > ps.have;
      for (int64_t r0 = 0; r0 < N; r0 += rows) {
        Task t{};
        t.type = k == 1 ? kBuild : kSpmm;
        t.slot = s;
        t.a = k;
        t.row0 = (int32_t)r0;
        t.row1 = (int32_t)std::min<int64_t>(r0 + rows, N);
        t.dep = dep ? counter(s, k - 1) : -1;
        t.dep_target = dep ? level_tasks[s][k - 1] : 0;
        t.done = counter(s, k);
        tasks.push_back(t);
        ++level_tasks[s][k];
      }
    }
    // every instance is queued at its level a (a >= 2 because m >= 3); when
    // that level is resident its trace has no dependency
    for (int j : by_level[k]) push_traces(j);
  }

  // staging (pinned) and device buffers
  const size_t tb = tasks.size() * sizeof(Task);
  size_t nptr = 0;
  for (int s = 0; s < nslots; ++s) nptr += c->sets[views[s].n].pw.size();
  TP_HIP_CHECK(grow_host(c->h_tasks, std::max<size_t>(tb, sizeof(Task))));
  TP_HIP_CHECK(grow_host(c->h_slots, kMaxSlots * sizeof(Slot)));
  TP_HIP_CHECK(grow_host(c->h_ptrs, std::max<size_t>(nptr, 1) * sizeof(void *)));
  TP_HIP_CHECK(grow_host(c->h_ctl, sizeof(Control)));
  TP_HIP_CHECK(grow(c->d_tasks, std::max<size_t>(tb, sizeof(Task))));
  TP_HIP_CHECK(grow(c->d_slots, kMaxSlots * sizeof(Slot)));
  TP_HIP_CHECK(grow(c->d_ptrs, std::max<size_t>(nptr, 1) * sizeof(void *)));
  TP_HIP_CHECK(grow(c->d_ctl, sizeof(Control)));
  TP_HIP_CHECK(grow(c->d_counters, (size_t)std::max(nslots * (kmax + 1), 1) * sizeof(int32_t)));
  TP_HIP_CHECK(grow(c->d_results, (size_t)std::max(count, 1) * sizeof(int32_t)));

  memcpy(c->h_tasks.p, tasks.data(), tb);
  Slot *hs = (Slot *)c->h_slots.p;
  void **hp = (void **)c->h_ptrs.p;
  size_t off = 0;
  for (int s = 0; s < nslots; ++s) {
    const PowerSet &ps = c->sets[views[s].n];
    Slot sl{};
    sl.n = views[s].n;
    sl.N = (int32_t)ps.N;
    sl.ld = ps.ld;
    sl.full = (1u << sl.n) - 1u;
    sl.masks = views[s].masks;
    sl.rowptr = views[s].rowptr;
    sl.col = views[s].col;
    sl.z = views[s].z;
    sl.powers = (uint16_t *const *)((void **)c->d_ptrs.p + off);
    hs[s] = sl;
    for (size_t k = 0; k < ps.pw.size(); ++k) hp[off + k] = ps.pw[k];
    off += ps.pw.size();
  }
  Control *hc = (Control *)c->h_ctl.p;
  hc->head = 0;
  hc->ntasks = (int32_t)tasks.size();
  hc->abort = 0;
  hc->pad = 0;
  hc->wait_limit = c->wait_limit;

  const int grid = c->grid_override > 0 ? c->grid_override : default_grid();
  if (!c->exec || c->g_key[0] != c->d_tasks.p || c->g_key[1] != c->d_counters.p ||
      c->g_key[2] != c->d_results.p || c->g_grid != grid ||
      c->g_counter_cap != c->d_counters.bytes || c->g_result_cap != c->d_results.bytes) {
    const int rc = capture_graph(c, grid);
    if (rc != TP_OK) return rc;
  }
  TP_HIP_CHECK(hipMemcpyAsync(c->d_tasks.p, c->h_tasks.p, tb, hipMemcpyHostToDevice, stream));
  TP_HIP_CHECK(hipMemcpyAsync(c->d_slots.p, c->h_slots.p, nslots * sizeof(Slot),
                              hipMemcpyHostToDevice, stream));
  TP_HIP_CHECK(hipMemcpyAsync(c->d_ptrs.p, c->h_ptrs.p, std::max<size_t>(nptr, 1) * sizeof(void *),
                              hipMemcpyHostToDevice, stream));
  TP_HIP_CHECK(hipMemcpyAsync(c->d_ctl.p, c->h_ctl.p, sizeof(Control), hipMemcpyHostToDevice,
                              stream));
  if (!c->staged) TP_HIP_CHECK(hipEventCreateWithFlags(&c->staged, hipEventDisableTiming));
  TP_HIP_CHECK(hipEventRecord(c->staged, stream));
  TP_HIP_CHECK(hipGraphLaunch(c->exec, stream));
  TP_HIP_CHECK(hipMemcpyAsync(gamma2_dev, c->d_results.p, (size_t)count * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, stream));
  // the levels just queued count as resident for later batches on this
  // stream; tp_ctx_check drops them again if the batch aborted
  c->pending = true;
  for (auto &kv : need) {
    PowerSet &ps = c->sets[kv.first];
    c->pending_n.push_back(kv.first);
    c->pending_have.push_back(ps.have);
    ps.have = std::max(ps.have, kv.second);
  }
  return TP_OK;
}

int ctx_check(Ctx *c, hipStream_t stream) {
  TP_HIP_CHECK(hipStreamSynchronize(stream));
  if (!c->pending) return TP_OK;
  c->pending = false;
  int32_t abort = 0;
  if (c->d_ctl.p)
    TP_HIP_CHECK(hipMemcpy(&abort, (char *)c->d_ctl.p + offsetof(Control, abort), sizeof(int32_t),
                           hipMemcpyDeviceToHost));
  if (abort) {
    // nothing computed by the aborted batches can be trusted
    for (size_t i = 0; i < c->pending_n.size(); ++i)
      c->sets[c->pending_n[i]].have = std::min(c->sets[c->pending_n[i]].have, c->pending_have[i]);
    c->pending_n.clear();
    c->pending_have.clear();
    set_error("batch aborted: a task waited longer than the limit for its inputs");
    return TP_ECANCELED;
  }
  c->pending_n.clear();
  c->pending_have.clear();
  return TP_OK;
}

void ctx_free(Ctx *c) {
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->staged) (void)hipEventDestroy(c->staged);
  for (auto &kv : c->sets)
    for (void *p : kv.second.pw) (void)hipFree(p);
  Buf *dev[] = {&c->d_tasks, &c->d_slots, &c->d_ptrs, &c->d_counters, &c->d_results, &c->d_ctl};
  for (Buf *b : dev)
    if (b->p) (void)hipFree(b->p);
  Buf *host[] = {&c->h_tasks, &c->h_slots, &c->h_ptrs, &c->h_ctl, &c->h_flag};
  for (Buf *b : host)
    if (b->p) (void)hipHostFree(b->p);
}

}  // namespace tp

using namespace tp;

extern "C" {

int tp_ctx_create(size_t hbm_budget_bytes, void **ctx) {
  TP_REQUIRE(ctx != nullptr, "ctx is NULL");
  Ctx *c = new Ctx();
  (void)hipGetDevice(&c->device);
  c->budget = hbm_budget_bytes;
  *ctx = c;
  return TP_OK;
}

int tp_ctx_destroy(void *ctx) {
  TP_REQUIRE(ctx != nullptr, "ctx is NULL");
  Ctx *c = (Ctx *)ctx;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    (void)hipDeviceSynchronize();
    ctx_free(c);
  }
  delete c;
  return TP_OK;
}

int tp_ctx_set_param(void *ctx, int param, int64_t value) {
  TP_REQUIRE(ctx != nullptr, "ctx is NULL");
  Ctx *c = (Ctx *)ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  switch (param) {
    case TP_PARAM_WAIT_LIMIT_US:
      TP_REQUIRE(value >= 0, "negative wait limit");
      c->wait_limit = value * 100;  // 100 MHz ticks
      return TP_OK;
    case TP_PARAM_GRID:
      TP_REQUIRE(value >= 0 && value <= (1 << 20), "grid out of range");
      c->grid_override = (int)value;
      return TP_OK;
    default:
      if (param >= TP_PARAM_SPMM_ROWS && param < TP_PARAM_SPMM_ROWS + 16) {
        TP_REQUIRE(value >= 0 && value <= 65536, "rows per task out of range");
        c->spmm_rows[param - TP_PARAM_SPMM_ROWS] = (int)(value + 3) / 4 * 4;
        return TP_OK;
      }
      set_error("unknown parameter %d", param);
      return TP_EINVAL;
  }
}

int64_t tp_ctx_resident_bytes(void *ctx) {
  if (!ctx) {
    set_error("ctx is NULL");
    return TP_EINVAL;
  }
  return (int64_t)((Ctx *)ctx)->used;
}

int tp_batch_power_trace(void *ctx, int count, const int32_t *n, const int64_t *m,
                         int32_t *gamma2_dev, hipStream_t stream) {
  TP_REQUIRE(ctx != nullptr, "ctx is NULL");
  TP_REQUIRE(count >= 0, "negative count");
  if (count == 0) return TP_OK;
  TP_REQUIRE(n && m && gamma2_dev, "NULL pointer");
  for (int j = 0; j < count; ++j) {
    TP_REQUIRE(n[j] >= 1 && n[j] <= 12, "instance %d: n = %d outside 1..12", j, n[j]);
    TP_REQUIRE(m[j] >= 3, "instance %d: m = %lld must be at least 3", j, (long long)m[j]);
    if ((int64_t)n[j] * m[j] >= 0xFFFF) {
      set_error("instance %d: n * m = %lld could reach INF", j, (long long)(n[j] * m[j]));
      return TP_EOVERFLOW;
    }
  }
  Ctx *c = (Ctx *)ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  return batch_run(c, count, n, m, gamma2_dev, stream);
}

int tp_ctx_check(void *ctx, hipStream_t stream) {
  TP_REQUIRE(ctx != nullptr, "ctx is NULL");
  Ctx *c = (Ctx *)ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  return ctx_check(c, stream);
}

}  // extern "C"
