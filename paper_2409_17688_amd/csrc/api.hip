// C ABI of libtropical.so: argument checks, the per-device cache of state
// matrices, and the schedule of tp_tropical_power_trace.
//
// gamma_2(P_n x C_m) = min_i (A^m)_ii (Theorem 2).  Every schedule below
// computes exactly that number, because the (min,+) semiring on integers is
// associative and exact:
//   * chain:  X <- A x X with the sparse left factor (Algorithm 2's order,
//             one pass costs nnz(A) * N operations instead of N^3);
//   * squaring: dense products P x P, P x Q of powers already formed;
//   * closing trace: min_{i,k} (A^a)_ik + (A^b)_ki gives the trace of A^(a+b)
//             without forming that product.
// Plan(c): chain to A^c (snapshotting A^r, r = m mod c, on the way), raise
// A^c to the q = m div c by square-and-multiply, and close with one trace of a
// product.  The planner prices every c with per-operation rates and picks the
// cheapest; c >= m/2 is a pure chain closed by one trace.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace tp {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int hip_fail(hipError_t e, const char *what) {
  set_error("%s failed: %s", what, hipGetErrorString(e));
  return TP_EHIP;
}

namespace {

bool valid_dtype(int dt) { return dt == TP_U8 || dt == TP_U16; }
size_t elem_size(int dt) { return dt == TP_U16 ? 2 : 1; }

// Device buffer owned by the cache.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
};

hipError_t ensure(DevBuf &b, size_t bytes) {
  if (b.bytes >= bytes && b.ptr) return hipSuccess;
  if (b.ptr) {
    hipError_t e = hipFree(b.ptr);
    if (e != hipSuccess) return e;
    b.ptr = nullptr;
    b.bytes = 0;
  }
  if (bytes == 0) return hipSuccess;
  hipError_t e = hipMalloc(&b.ptr, bytes);
  if (e == hipSuccess) b.bytes = bytes;
  return e;
}

void release(DevBuf &b) {
  if (b.ptr) (void)hipFree(b.ptr);
  b.ptr = nullptr;
  b.bytes = 0;
}

// Per (device, n): word masks, zero counts and the CSR of A(D_n).
struct State {
  int n = 0;
  int64_t N = 0, nnz = -1;
  DevBuf masks, z, rowptr, col, colz;
  DevBuf bptr, bent;  // blocked form of A(D_n), 16 rows per block
  DevBuf order;       // rows by decreasing out-degree (int32), for the packed gather
  DevBuf border;      // row blocks by decreasing entry count (int32), for the blocked step
  int64_t nent = 0;
  bool csr_ready = false;
  std::vector<uint8_t> zh;                // zero counts on the host
  std::vector<int32_t> degh;              // out-degrees on the host
  std::map<int, DevBuf> sel;              // states with <= k zeros (device int32), by k
  std::map<int, int64_t> sel_count;
  // row blocks cut by rows into parts (the small-n step, the batch kernel's
  // chain levels)
  DevBuf fptr, fent, finfo, forder;
  std::vector<int64_t> fptrh;
  bool fine_ready = false;
};

struct Workspace {
  DevBuf buf[6];
  DevBuf scalar;  // int32 results
};

std::mutex g_mu;
std::map<std::pair<int, int>, State> g_states;  // (device, n)
std::map<int, Workspace> g_ws;                  // device

int current_device() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}

int build_fine(State &st, hipStream_t s);

// The parts of a state as the step launchers take them (nf = 0: not built).
FineView fine_of(const State &st) {
  FineView f{};
  if (!st.fine_ready) return f;
  f.nf = (int64_t)st.fptrh.size() - 1;
  f.fptr = (const int64_t *)st.fptr.ptr;
  f.fent = (const uint64_t *)st.fent.ptr;
  f.finfo = (const uint32_t *)st.finfo.ptr;
  f.forder = (const int32_t *)st.forder.ptr;
  f.fptrh = st.fptrh.data();
  return f;
}

// Builds masks, zero counts and the CSR of A(D_n) on `s` (blocking only
// for the arc count, which sizes the column array), and for n <= 10 the
// row-block parts of the small-n step.  Caller holds g_mu.
int get_state(int n, hipStream_t s, State **out) {
  State &st = g_states[{current_device(), n}];
  if (!st.csr_ready) {
    st.n = n;
    st.N = word_count_host(n);
    const int64_t N = st.N;
    TP_HIP_CHECK(ensure(st.masks, N * sizeof(uint32_t)));
    TP_HIP_CHECK(ensure(st.z, N));
    TP_HIP_CHECK(ensure(st.rowptr, (N + 1) * sizeof(int64_t)));
    TP_HIP_CHECK(launch_words(n, nullptr, (uint8_t *)st.z.ptr, (uint32_t *)st.masks.ptr, s));
    TP_HIP_CHECK(launch_csr_count(N, n, (const uint32_t *)st.masks.ptr, (int64_t *)st.rowptr.ptr, s));
    TP_HIP_CHECK(launch_scan_rowptr(N, (int64_t *)st.rowptr.ptr, s));
    int64_t nnz = 0;
    TP_HIP_CHECK(hipMemcpyAsync(&nnz, (int64_t *)st.rowptr.ptr + N, sizeof(int64_t),
                                hipMemcpyDeviceToHost, s));
    TP_HIP_CHECK(hipStreamSynchronize(s));
    st.nnz = nnz;
    TP_HIP_CHECK(ensure(st.col, (size_t)nnz * sizeof(uint32_t)));
    TP_HIP_CHECK(ensure(st.colz, (size_t)nnz * sizeof(uint32_t)));
    TP_HIP_CHECK(launch_csr_fill(N, n, (const uint32_t *)st.masks.ptr,
                                 (const int64_t *)st.rowptr.ptr, (uint32_t *)st.col.ptr,
                                 (uint32_t *)st.colz.ptr, s));
    const int64_t nb = block_count_host(N);
    TP_HIP_CHECK(ensure(st.bptr, (nb + 1) * sizeof(int64_t)));
    TP_HIP_CHECK(launch_block_count(N, n, (const uint32_t *)st.masks.ptr, (int64_t *)st.bptr.ptr, s));
    TP_HIP_CHECK(launch_scan_rowptr(nb, (int64_t *)st.bptr.ptr, s));
    int64_t nent = 0;
    TP_HIP_CHECK(hipMemcpyAsync(&nent, (int64_t *)st.bptr.ptr + nb, sizeof(int64_t),
                                hipMemcpyDeviceToHost, s));
    TP_HIP_CHECK(hipStreamSynchronize(s));
    st.nent = nent;
    TP_HIP_CHECK(ensure(st.bent, (size_t)std::max<int64_t>(nent, 1) * sizeof(uint64_t)));
    TP_HIP_CHECK(launch_block_fill(N, n, (const uint32_t *)st.masks.ptr,
                                   (const int64_t *)st.bptr.ptr, (uint64_t *)st.bent.ptr, s));
    {
      // the blocked step's order: blocks with the most entries first
      std::vector<int64_t> bp((size_t)nb + 1);
      TP_HIP_CHECK(hipMemcpyAsync(bp.data(), st.bptr.ptr, bp.size() * sizeof(int64_t),
                                  hipMemcpyDeviceToHost, s));
      TP_HIP_CHECK(hipStreamSynchronize(s));
      // within each block, entries grouped by their row mask (then by p),
      // the last entry of each group flagged in bit 48: rows with the same
      // successors take one combined minimum per group (the grouped step);
      // every other reader ignores the order and bit 48
      if (nent > 0) {
        std::vector<uint64_t> e((size_t)nent);
        TP_HIP_CHECK(hipMemcpyAsync(e.data(), st.bent.ptr, e.size() * sizeof(uint64_t),
                                    hipMemcpyDeviceToHost, s));
        TP_HIP_CHECK(hipStreamSynchronize(s));
        // groups in the order of their least successor, so a block still
        // sweeps X roughly by increasing row (the rows it gathers come from
        // HBM in fewer, longer runs)
        auto key = [](uint64_t x) { return ((x >> 32) & 0xFFFFull) << 24 | (x & 0xFFFFFFull); };
        std::vector<uint64_t> tmp;
        std::vector<std::pair<uint64_t, int64_t>> runs;  // (least p, start), then its end
        for (int64_t b = 0; b < nb; ++b) {
          auto first = e.begin() + bp[b], last = e.begin() + bp[b + 1];
          std::sort(first, last, [&](uint64_t a, uint64_t c) { return key(a) < key(c); });
          runs.clear();
          for (int64_t i = bp[b]; i < bp[b + 1]; ++i)
            if (i == bp[b] || ((e[i - 1] ^ e[i]) >> 32 & 0xFFFFull) != 0)
              runs.push_back({e[i] & 0xFFFFFFull, i});
          std::vector<int64_t> ends(runs.size());
          for (size_t g = 0; g < runs.size(); ++g)
            ends[g] = g + 1 < runs.size() ? runs[g + 1].second : bp[b + 1];
          std::vector<size_t> ord(runs.size());
          for (size_t g = 0; g < ord.size(); ++g) ord[g] = g;
          std::sort(ord.begin(), ord.end(),
                    [&](size_t a, size_t c) { return runs[a].first < runs[c].first; });
          tmp.clear();
          for (size_t g : ord) {
            for (int64_t i = runs[g].second; i < ends[g]; ++i) tmp.push_back(e[i]);
            tmp.back() |= kGroupEnd;
          }
          std::copy(tmp.begin(), tmp.end(), first);
        }
        TP_HIP_CHECK(hipMemcpyAsync(st.bent.ptr, e.data(), e.size() * sizeof(uint64_t),
                                    hipMemcpyHostToDevice, s));
        TP_HIP_CHECK(hipStreamSynchronize(s));
      }
      std::vector<int32_t> bo((size_t)nb);
      for (int64_t b = 0; b < nb; ++b) bo[b] = (int32_t)b;
      std::stable_sort(bo.begin(), bo.end(), [&](int32_t a, int32_t c) {
        return bp[a + 1] - bp[a] > bp[c + 1] - bp[c];
      });
      TP_HIP_CHECK(ensure(st.border, std::max<size_t>(bo.size(), 1) * sizeof(int32_t)));
      // on the call's stream: a synchronous copy would wait for the work
      // other streams have in flight
      if (nb > 0) {
        TP_HIP_CHECK(hipMemcpyAsync(st.border.ptr, bo.data(), bo.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, s));
        TP_HIP_CHECK(hipStreamSynchronize(s));
      }
    }
    st.zh.assign((size_t)N, 0);
    TP_HIP_CHECK(hipMemcpyAsync(st.zh.data(), st.z.ptr, (size_t)N, hipMemcpyDeviceToHost, s));
    // the gather's row order: longest successor lists first, so that the
    // longest chains of dependent gathers start with the launch instead of
    // ending it (the all-zero word alone has 2^n successors)
    std::vector<int64_t> rp((size_t)N + 1);
    TP_HIP_CHECK(hipMemcpyAsync(rp.data(), st.rowptr.ptr, rp.size() * sizeof(int64_t),
                                hipMemcpyDeviceToHost, s));
    TP_HIP_CHECK(hipStreamSynchronize(s));
    std::vector<int32_t> ord((size_t)N);
    st.degh.assign((size_t)N, 0);
    for (int64_t i = 0; i < N; ++i) {
      ord[i] = (int32_t)i;
      st.degh[i] = (int32_t)(rp[i + 1] - rp[i]);
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
      return rp[a + 1] - rp[a] > rp[b + 1] - rp[b];
    });
    TP_HIP_CHECK(ensure(st.order, std::max<size_t>(ord.size(), 1) * sizeof(int32_t)));
    if (N > 0) {
      TP_HIP_CHECK(hipMemcpyAsync(st.order.ptr, ord.data(), ord.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, s));
      TP_HIP_CHECK(hipStreamSynchronize(s));
    }
    st.csr_ready = true;
    if (n <= 10) {
      const int rc = build_fine(st, s);
      if (rc != TP_OK) return rc;
    }
  }
  *out = &st;
  return TP_OK;
}

// ---------------------------------------------------------------- planner --

// Kernel rates by path order n (rows padded to 64 entries): (min,+)
// operations per second of one sparse left step (nnz * N operations) and of
// one dense product (N^3), plus launch overhead.  The defaults were measured
// on an MI355X; the autotuner replaces them (tp_tune_planner).  Only their
// ratios steer the plan; every plan gives the same answer.  Guarded by g_mu.
constexpr double kSpmmRate[13] = {0, 1e10, 1e10, 2e10, 5e10, 1e11, 5e10, 2.5e11,
                                  1.4e12, 4.5e12, 1.19e13, 1.05e13, 1.12e13};
constexpr double kGemmRate[13] = {0, 1e9, 1e9, 1e10, 5e10, 1e11, 3e11, 2e12,
                                  1.45e13, 2.6e13, 3.37e13, 3.4e13, 3.4e13};
double g_spmm_rate[13] = {0, 1e10, 1e10, 2e10, 5e10, 1e11, 5e10, 2.5e11,
                          1.4e12, 4.5e12, 1.19e13, 1.05e13, 1.12e13};
double g_gemm_rate[13] = {0, 1e9, 1e9, 1e10, 5e10, 1e11, 3e11, 2e12,
                          1.45e13, 2.6e13, 3.37e13, 3.4e13, 3.4e13};
// Form of the sparse left step by n when TP_STEP_AUTO is asked for (0: the
// built-in rule, row blocks taken a mask group at a time from n = 8 on,
// where they were measured faster: n = 12 40.7 ms against 101 ms for the
// per-row gather, n = 10 0.51 against 0.92 ms, n = 9 0.057 against 0.104 ms
// and n = 8 21 against 27 us with a workgroup's waves sharing each block;
// the gather wins below).
// Guarded by g_mu.
int g_step_form[14] = {0};  // n = 1..13

int step_form(int n, int form) {
  if (form != TP_STEP_AUTO) return form;
  if (g_step_form[n] != TP_STEP_AUTO) return g_step_form[n];
  return n >= 8 ? TP_STEP_BLOCKED : TP_STEP_CSR;
}

// Y = A(D_n) x X (u16) with the state's CSR or blocked form.  Caller holds g_mu.
hipError_t state_step(const State *st, int form, const uint16_t *X, int64_t ldx, uint16_t *Y,
                      int64_t ldy, int64_t ncols, hipStream_t s) {
  const int f = step_form(st->n, form);
  if (f == TP_STEP_BLOCKED || f == TP_STEP_BLOCKED_ENTRIES) {
    const FineView fine = fine_of(*st);
    return launch_block_step(st->N, (const int64_t *)st->bptr.ptr,
                             (const uint64_t *)st->bent.ptr, (const int32_t *)st->border.ptr,
                             &fine, X, ldx, Y, ldy, ncols, f == TP_STEP_BLOCKED, s);
  }
  if (state_gather_fits(X, ldx, Y, ldy, ncols))
    return launch_state_gather(st->N, (const int64_t *)st->rowptr.ptr,
                               (const uint32_t *)st->colz.ptr, (const int32_t *)st->order.ptr, X,
                               ldx, Y, ldy, ncols, s);
  return launch_spmm(TP_U16, st->N, (const int64_t *)st->rowptr.ptr,
                     (const uint32_t *)st->col.ptr, (const uint8_t *)st->z.ptr, X, ldx, Y, ldy,
                     ncols, s);
}

constexpr double kHbm = 5.0e12;     // bytes / s for traces and copies
constexpr double kLaunch = 6.0e-6;  // s per kernel launch

int bit_length(int64_t v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}
int popcount64(int64_t v) { return __builtin_popcountll((unsigned long long)v); }

// products needed by left-to-right square-and-multiply to form P^q from P
int64_t sqm_products(int64_t q) { return q <= 1 ? 0 : (bit_length(q) - 1) + (popcount64(q) - 1); }

struct Plan {
  int64_t c = 1;        // chain length
  double cost = 1e300;  // estimated seconds
};

double plan_cost(int n, int64_t m, int64_t c, double N, double nnz) {
  const double S = nnz * N / g_spmm_rate[n] + kLaunch;
  const double G = N * N * N / g_gemm_rate[n] + kLaunch;
  const double T = 4.0 * N * N / kHbm + 2 * kLaunch;  // trace of a product, u16
  const double copy = 4.0 * N * N / kHbm + kLaunch;
  const int64_t q = m / c, r = m % c;
  double cost = (double)(c - 1) * S + N * N * 2.0 / kHbm;  // chain + dense start
  if (r > 0) {
    cost += copy + (double)sqm_products(q) * G + T;
  } else if (q == 1) {
    cost += N / kHbm + kLaunch;  // diagonal of A^m
  } else {
    const int64_t h = q / 2;
    cost += (double)sqm_products(h) * G + ((q & 1) ? G : 0.0) + T;
  }
  return cost;
}

Plan choose_plan(int n, int64_t m, double N, double nnz) {
  Plan best;
  for (int64_t c = 1; c <= m; ++c) {
    const double cst = plan_cost(n, m, c, N, nnz);
    if (cst < best.cost) {
      best.cost = cst;
      best.c = c;
    }
  }
  return best;
}

// Square-and-multiply: dst = P^q (q >= 1), P untouched; uses tmp.  Returns
// the buffer that holds the result (dst or P itself when q == 1).
int power_of(uint16_t *P, int64_t q, int64_t N, int64_t ld, uint16_t *dst, uint16_t *tmp,
             hipStream_t s, uint16_t **result) {
  if (q == 1) {
    *result = P;
    return TP_OK;
  }
  // left to right over the bits of q below the top one
  const int top = bit_length(q) - 1;
  uint16_t *cur = P;
  uint16_t *bufs[2] = {dst, tmp};
  int which = 0;
  for (int b = top - 1; b >= 0; --b) {
    uint16_t *o = bufs[which];
    TP_HIP_CHECK(launch_gemm(TP_U16, N, N, N, cur, ld, cur, ld, o, ld, 0, -1, -1, s));
    cur = o;
    which ^= 1;
    if ((q >> b) & 1) {
      uint16_t *o2 = bufs[which];
      TP_HIP_CHECK(launch_gemm(TP_U16, N, N, N, cur, ld, P, ld, o2, ld, 0, -1, -1, s));
      cur = o2;
      which ^= 1;
    }
  }
  *result = cur;
  return TP_OK;
}

// Pruning of start states: 0 = by the cost model, 1 = whenever valid, -1 =
// never (tp_tune_prune).  Guarded by g_mu.
int g_prune = 0;

int64_t count_selected(const State *st, int k) {
  int64_t c = 0;
  for (uint8_t z : st->zh) c += z <= k;
  return c;
}

// Device list of the states with at most k zeros, in increasing index (cached
// per k).  Caller holds g_mu.
int state_selection(State *st, int k, hipStream_t s, const int32_t **idx, int64_t *count) {
  auto it = st->sel_count.find(k);
  if (it == st->sel_count.end()) {
    std::vector<int32_t> h;
    for (size_t i = 0; i < st->zh.size(); ++i)
      if (st->zh[i] <= k) h.push_back((int32_t)i);
    DevBuf &b = st->sel[k];
    TP_HIP_CHECK(ensure(b, std::max<size_t>(h.size(), 1) * sizeof(int32_t)));
    if (!h.empty())
      TP_HIP_CHECK(hipMemcpyAsync(b.ptr, h.data(), h.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, s));
    TP_HIP_CHECK(hipStreamSynchronize(s));
    it = st->sel_count.emplace(k, (int64_t)h.size()).first;
  }
  *idx = (const int32_t *)st->sel[k].ptr;
  *count = it->second;
  return TP_OK;
}

// First guess of floor(gamma_2 / m): the walk label grows by about (n + 2) / 3
// per step for every n the paper tabulates; a wrong guess costs a second
// pass, never a wrong answer.
int prune_guess(int n) { return n >= 2 ? (n + 2) / 3 : 1; }

// gamma_2 as min over the states with at most k zeros of (A^m)_ii: the chain
// A^k e_i for those columns only.  Buffers 0 and 1 of the workspace.
int pruned_chain(State *st, int64_t m, int k, hipStream_t s, int32_t *out_host) {
  const int32_t *idx = nullptr;
  int64_t cnt = 0;
  int rc = state_selection(st, k, s, &idx, &cnt);
  if (rc != TP_OK) return rc;
  if (cnt == 0) {
    *out_host = kInf16;
    return TP_OK;
  }
  const int64_t N = st->N, ld = (cnt + 63) / 64 * 64;
  Workspace &ws = g_ws[current_device()];
  const size_t mat = (size_t)N * (size_t)ld * sizeof(uint16_t);
  TP_HIP_CHECK(ensure(ws.buf[0], mat));
  TP_HIP_CHECK(ensure(ws.buf[1], mat));
  TP_HIP_CHECK(ensure(ws.scalar, 64));
  uint16_t *X = (uint16_t *)ws.buf[0].ptr, *Y = (uint16_t *)ws.buf[1].ptr;
  int32_t *d_res = (int32_t *)ws.scalar.ptr;
  TP_HIP_CHECK(launch_state_columns(st->n, N, (const uint32_t *)st->masks.ptr, idx, cnt, X, ld, s));
  // from n = 11 on (tp_tune_compact_chains) the steps after A^3 run on
  // shared-base compact powers held in the same two buffers (u8 rows of ld
  // bytes), and the last power comes back to 16 bits for the diagonal
  constexpr int64_t kSwitch = 3;
  if (compact_chain(st->n) && m >= kSwitch + 2) {
    for (int64_t t = 2; t <= kSwitch; ++t) {
      TP_HIP_CHECK(state_step(st, TP_STEP_AUTO, X, ld, Y, ld, cnt, s));
      std::swap(X, Y);
    }
    int32_t *bx = d_res + 4, *by = d_res + 8, *status = d_res + 12;
    uint8_t *X8 = (uint8_t *)Y, *Y8 = (uint8_t *)X;  // Y8 overwrites the 16-bit A^3 after it is read
    TP_HIP_CHECK(launch_fill_i32(status, 1, 0, s));
    TP_HIP_CHECK(launch_shared_from_u16(N, cnt, X, ld, X8, ld, bx, status, s));
    StateView v{};
    v.n = st->n;
    v.N = N;
    v.bptr = (const int64_t *)st->bptr.ptr;
    v.bent = (const uint64_t *)st->bent.ptr;
    v.border = (const int32_t *)st->border.ptr;
    for (int64_t t = kSwitch + 1; t <= m; ++t) {
      TP_HIP_CHECK(launch_shared_step(v, X8, ld, bx, Y8, ld, by, cnt, status, s));
      std::swap(X8, Y8);
      std::swap(bx, by);
    }
    // the last power (in X8) to 16 bits in the other buffer
    uint16_t *P = (uint16_t *)Y8;
    TP_HIP_CHECK(launch_shared_to_u16(N, cnt, X8, ld, bx, P, ld, s));
    TP_HIP_CHECK(launch_diag_select_min(N, cnt, idx, P, ld, d_res, s));
    int32_t host[13] = {0};
    TP_HIP_CHECK(hipMemcpyAsync(host, d_res, sizeof(host), hipMemcpyDeviceToHost, s));
    TP_HIP_CHECK(hipStreamSynchronize(s));
    if (host[12] == 0) {
      *out_host = host[0];
      return TP_OK;
    }
    // a power the compact form could not hold: the 16-bit chain from the start
    TP_HIP_CHECK(launch_state_columns(st->n, N, (const uint32_t *)st->masks.ptr, idx, cnt, X, ld,
                                      s));
  }
  for (int64_t t = 2; t <= m; ++t) {
    TP_HIP_CHECK(state_step(st, TP_STEP_AUTO, X, ld, Y, ld, cnt, s));
    std::swap(X, Y);
  }
  TP_HIP_CHECK(launch_diag_select_min(N, cnt, idx, X, ld, d_res, s));
  TP_HIP_CHECK(hipMemcpyAsync(out_host, d_res, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  TP_HIP_CHECK(hipStreamSynchronize(s));
  return TP_OK;
}

// The pruned chain with the guessed bound, then, if the value found allows
// states with more zeros (floor(value / m) above the guess), once more with
// that bound, which then covers the optimal walk's start.
int pruned_power_trace(State *st, int64_t m, hipStream_t s, int32_t *gamma2_host) {
  const int k1 = prune_guess(st->n);
  int32_t g = 0;
  int rc = pruned_chain(st, m, k1, s, &g);
  if (rc != TP_OK) return rc;
  const int64_t k2 = g / m;
  if (k2 > k1) {
    int32_t g2 = 0;
    rc = pruned_chain(st, m, (int)std::min<int64_t>(k2, st->n), s, &g2);
    if (rc != TP_OK) return rc;
    g = std::min(g, g2);
  }
  *gamma2_host = g;
  return TP_OK;
}

int power_trace_locked(int n, int64_t m, int32_t *gamma2_host, hipStream_t s) {
  State *st = nullptr;
  int rc = get_state(n, s, &st);
  if (rc != TP_OK) return rc;
  const int64_t N = st->N;
  Workspace &ws = g_ws[current_device()];
  // rows padded to 64 entries (128 bytes) so every row starts aligned for
  // 16-byte loads whatever N is
  const int64_t ld = (N + 63) / 64 * 64;
  const size_t mat = (size_t)N * (size_t)ld * sizeof(uint16_t);
  const Plan plan = choose_plan(n, m, (double)N, (double)st->nnz);
  if (g_prune >= 0) {
    // pruned chain: m - 1 sparse steps on |S| columns, one selected diagonal.
    // A step on the narrow panel runs at about 3/4 of the full step's rate,
    // and up to n = 10 no faster than 0.65 of a full step (latency of the
    // gathered rows); measured so, it wins from n = 12 on (1.25-1.35x).
    const double cnt = (double)count_selected(st, prune_guess(n));
    const double full = (double)st->nnz * (double)N / g_spmm_rate[n] + kLaunch;
    const double step = std::max(full * (cnt / (double)N) / 0.75, n <= 10 ? 0.65 * full : 0.0);
    const double cost = (double)(m - 1) * step + 2.0 * N * cnt / kHbm;
    if (g_prune > 0 || cost < plan.cost) return pruned_power_trace(st, m, s, gamma2_host);
  }
  const int64_t c = plan.c, q = m / c, r = m % c;

  TP_HIP_CHECK(ensure(ws.scalar, 64));
  int32_t *d_res = (int32_t *)ws.scalar.ptr;
  // buffers: 0,1 chain ping-pong; 2 snapshot A^r; 3,4 powering; 5 spare
  const int pw = r > 0 ? 3 : 2;
  const int needed = pw + (q > 1 ? 2 : 0);
  for (int i = 0; i < needed; ++i) TP_HIP_CHECK(ensure(ws.buf[i], mat));
  uint16_t *X = (uint16_t *)ws.buf[0].ptr, *Y = (uint16_t *)ws.buf[1].ptr;
  uint16_t *snap = r > 0 ? (uint16_t *)ws.buf[2].ptr : nullptr;

  // X = A^1, then the chain up to A^c
  const uint32_t *masks = (const uint32_t *)st->masks.ptr;
  TP_HIP_CHECK(launch_dense_state(n, N, masks, TP_U16, X, ld, s));
  if (r == 1) TP_HIP_CHECK(hipMemcpyAsync(snap, X, mat, hipMemcpyDeviceToDevice, s));
  for (int64_t k = 2; k <= c; ++k) {
    TP_HIP_CHECK(state_step(st, TP_STEP_AUTO, X, ld, Y, ld, N, s));
    uint16_t *t = X;
    X = Y;
    Y = t;
    if (k == r) TP_HIP_CHECK(hipMemcpyAsync(snap, X, mat, hipMemcpyDeviceToDevice, s));
  }
  // X = A^c
  if (r > 0) {
    uint16_t *R = nullptr;
    rc = power_of(X, q, N, ld, (uint16_t *)ws.buf[pw].ptr, (uint16_t *)ws.buf[pw + 1].ptr, s, &R);
    if (rc != TP_OK) return rc;
    TP_HIP_CHECK(launch_trace_of_product(TP_U16, N, R, ld, snap, ld, d_res, s));
  } else if (q == 1) {
    TP_HIP_CHECK(launch_trace_min(TP_U16, N, X, ld, d_res, s));
  } else {
    const int64_t h = q / 2;
    uint16_t *H = nullptr;
    uint16_t *tmp_a = (uint16_t *)ws.buf[pw].ptr, *tmp_b = (uint16_t *)ws.buf[pw + 1].ptr;
    rc = power_of(X, h, N, ld, tmp_a, tmp_b, s, &H);
    if (rc != TP_OK) return rc;
    if (q & 1) {
      // H x X = P^(h+1) into a buffer that is neither H nor X
      uint16_t *o = (H == tmp_a) ? tmp_b : tmp_a;
      if (H == X) o = tmp_a;
      TP_HIP_CHECK(launch_gemm(TP_U16, N, N, N, H, ld, X, ld, o, ld, 0, -1, -1, s));
      TP_HIP_CHECK(launch_trace_of_product(TP_U16, N, H, ld, o, ld, d_res, s));
    } else {
      TP_HIP_CHECK(launch_trace_of_product(TP_U16, N, H, ld, H, ld, d_res, s));
    }
  }
  int32_t host = 0;
  TP_HIP_CHECK(hipMemcpyAsync(&host, d_res, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  TP_HIP_CHECK(hipStreamSynchronize(s));
  *gamma2_host = host;
  return TP_OK;
}

}  // namespace

void step_and_product_seconds(int n, double N, double nnz, double *step, double *product) {
  std::lock_guard<std::mutex> lk(g_mu);
  *step = nnz * N / g_spmm_rate[n] + kLaunch;
  *product = N * N * N / g_gemm_rate[n] + kLaunch;
}

hipError_t state_step_view(const StateView &v, const uint16_t *X, int64_t ldx, uint16_t *Y,
                           int64_t ldy, int64_t ncols, hipStream_t s) {
  int form;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    form = step_form(v.n, TP_STEP_AUTO);
  }
  if (form == TP_STEP_BLOCKED || form == TP_STEP_BLOCKED_ENTRIES)
    return launch_block_step(v.N, v.bptr, v.bent, v.border, &v.fine, X, ldx, Y, ldy, ncols,
                             form == TP_STEP_BLOCKED, s);
  if (state_gather_fits(X, ldx, Y, ldy, ncols))
    return launch_state_gather(v.N, v.rowptr, v.colz, v.order, X, ldx, Y, ldy, ncols, s);
  return launch_spmm(TP_U16, v.N, v.rowptr, v.col, v.z, X, ldx, Y, ldy, ncols, s);
}

namespace {

// Parts of the row blocks, for the steps that give each (part, 256-column
// panel) to one workgroup, whose waves split the part's entries, so the
// longest part bounds the step.  A block with more than T entries is cut
// into runs of consecutive rows, each run as long as its successors' union
// stays within T (a single row with more successors is a part of its own);
// a part keeps the block's entries that reach its rows, with their masks cut
// to those rows and grouped again by mask.  T is half the longest block (at
// least 128) up to n = 8, where the stand-alone step gives each part a
// workgroup: the longest runs of entries halve, for about a third more
// entries in all (the rows of a block share most successors).  From n = 9
// only the fused batch levels take parts, whose workgroups draw the next
// item when free; there three quarters of the longest block gather less
// (225 parts of 1.04x the block entries at n = 9 against 284 of 1.28x)
// and ran the mixed 64-instance batch 3 - 5 % faster.
int build_fine(State &st, hipStream_t s) {
  const int64_t N = st.N, nb = (N + 15) / 16, nent = st.nent;
  std::vector<int64_t> bp((size_t)nb + 1);
  std::vector<uint64_t> e((size_t)std::max<int64_t>(nent, 1));
  TP_HIP_CHECK(hipMemcpyAsync(bp.data(), st.bptr.ptr, bp.size() * sizeof(int64_t),
                              hipMemcpyDeviceToHost, s));
  if (nent > 0)
    TP_HIP_CHECK(hipMemcpyAsync(e.data(), st.bent.ptr, (size_t)nent * sizeof(uint64_t),
                                hipMemcpyDeviceToHost, s));
  TP_HIP_CHECK(hipStreamSynchronize(s));
  int64_t longest = 0;
  for (int64_t b = 0; b < nb; ++b) longest = std::max(longest, bp[b + 1] - bp[b]);
  const int64_t T = std::max<int64_t>(128, st.n >= 9 ? longest * 3 / 4 : longest / 2);
  std::vector<int64_t> fp(1, 0);
  std::vector<uint64_t> fe;
  std::vector<uint32_t> fi;
  std::vector<uint64_t> tmp;
  auto mask_of = [](uint64_t x) { return (uint32_t)((x >> 32) & 0xFFFFull); };
  auto emit = [&](int64_t b, uint32_t part) {
    // the block's entries that reach these rows, masks cut to them, grouped
    // by mask (groups in the order of their least successor)
    tmp.clear();
    for (int64_t i = bp[b]; i < bp[b + 1]; ++i) {
      const uint32_t m = mask_of(e[i]) & part;
      if (m) tmp.push_back((e[i] & 0xFFFFFFFFull) | ((uint64_t)m << 32));
    }
    std::sort(tmp.begin(), tmp.end(), [&](uint64_t a, uint64_t c) {
      const uint64_t ka = (uint64_t)mask_of(a) << 24 | (a & 0xFFFFFFull);
      const uint64_t kc = (uint64_t)mask_of(c) << 24 | (c & 0xFFFFFFull);
      return ka < kc;
    });
    std::vector<std::pair<uint64_t, size_t>> runs;  // (least p, start)
    for (size_t i = 0; i < tmp.size(); ++i)
      if (i == 0 || mask_of(tmp[i - 1]) != mask_of(tmp[i])) runs.push_back({tmp[i] & 0xFFFFFFull, i});
    std::sort(runs.begin(), runs.end());
    for (size_t g = 0; g < runs.size(); ++g) {
      const uint32_t m = mask_of(tmp[runs[g].second]);
      size_t i = runs[g].second;
      for (; i < tmp.size() && mask_of(tmp[i]) == m; ++i) fe.push_back(tmp[i]);
      fe.back() |= kGroupEnd;
    }
    fp.push_back((int64_t)fe.size());
    fi.push_back((uint32_t)(b << 16) | part);
  };
  for (int64_t b = 0; b < nb; ++b) {
    const int rows = (int)std::min<int64_t>(16, N - b * 16);
    const uint32_t all = (1u << rows) - 1u;
    if (bp[b + 1] - bp[b] <= T) {
      emit(b, all);
      continue;
    }
    auto reach = [&](uint32_t part) {
      int64_t c = 0;
      for (int64_t i = bp[b]; i < bp[b + 1]; ++i) c += (mask_of(e[i]) & part) != 0;
      return c;
    };
    uint32_t cur = 0;
    for (int r = 0; r < rows; ++r) {
      const uint32_t cand = cur | (1u << r);
      if (cur != 0 && reach(cand) > T) {
        emit(b, cur);
        cur = 1u << r;
      } else {
        cur = cand;
      }
    }
    if (cur) emit(b, cur);
  }
  const int64_t nf = (int64_t)fi.size();
  std::vector<int32_t> fo((size_t)nf);
  for (int64_t f = 0; f < nf; ++f) fo[f] = (int32_t)f;
  std::stable_sort(fo.begin(), fo.end(), [&](int32_t a, int32_t c) {
    return fp[a + 1] - fp[a] > fp[c + 1] - fp[c];
  });
  TP_HIP_CHECK(ensure(st.forder, std::max<size_t>(fo.size(), 1) * sizeof(int32_t)));
  TP_HIP_CHECK(ensure(st.fptr, fp.size() * sizeof(int64_t)));
  TP_HIP_CHECK(ensure(st.fent, std::max<size_t>(fe.size(), 1) * sizeof(uint64_t)));
  TP_HIP_CHECK(ensure(st.finfo, std::max<size_t>(fi.size(), 1) * sizeof(uint32_t)));
  TP_HIP_CHECK(hipMemcpyAsync(st.fptr.ptr, fp.data(), fp.size() * sizeof(int64_t),
                              hipMemcpyHostToDevice, s));
  if (!fe.empty())
    TP_HIP_CHECK(hipMemcpyAsync(st.fent.ptr, fe.data(), fe.size() * sizeof(uint64_t),
                                hipMemcpyHostToDevice, s));
  if (nf > 0) {
    TP_HIP_CHECK(hipMemcpyAsync(st.finfo.ptr, fi.data(), fi.size() * sizeof(uint32_t),
                                hipMemcpyHostToDevice, s));
    TP_HIP_CHECK(hipMemcpyAsync(st.forder.ptr, fo.data(), fo.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, s));
  }
  TP_HIP_CHECK(hipStreamSynchronize(s));
  st.fptrh = std::move(fp);
  st.fine_ready = true;
  return TP_OK;
}

}  // namespace

int state_fine_view(int n, hipStream_t s, FineView *out) {
  std::lock_guard<std::mutex> lk(g_mu);
  State *st = nullptr;
  int rc = get_state(n, s, &st);
  if (rc != TP_OK) return rc;
  if (!st->fine_ready) {
    rc = build_fine(*st, s);
    if (rc != TP_OK) return rc;
  }
  *out = fine_of(*st);
  return TP_OK;
}

int state_view(int n, hipStream_t s, StateView *out) {
  std::lock_guard<std::mutex> lk(g_mu);
  State *st = nullptr;
  const int rc = get_state(n, s, &st);
  if (rc != TP_OK) return rc;
  out->n = n;
  out->N = st->N;
  out->nnz = st->nnz;
  out->masks = (const uint32_t *)st->masks.ptr;
  out->rowptr = (const int64_t *)st->rowptr.ptr;
  out->col = (const uint32_t *)st->col.ptr;
  out->z = (const uint8_t *)st->z.ptr;
  out->colz = (const uint32_t *)st->colz.ptr;
  out->bptr = (const int64_t *)st->bptr.ptr;
  out->bent = (const uint64_t *)st->bent.ptr;
  out->nent = st->nent;
  out->order = (const int32_t *)st->order.ptr;
  out->border = (const int32_t *)st->border.ptr;
  out->degh = st->degh.data();
  out->fine = fine_of(*st);
  return TP_OK;
}

}  // namespace tp

using namespace tp;

extern "C" {

const char *tp_last_error(void) { return g_err; }

int tp_version(void) { return 1; }

int64_t tp_state_dim(int n) {
  if (n < 1 || n > 13) {
    set_error("n = %d outside 1..13", n);
    return TP_EINVAL;
  }
  return word_count_host(n);
}

int64_t tp_state_nnz(int n) {
  if (n < 1 || n > 13) {
    set_error("n = %d outside 1..13", n);
    return TP_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  State *st = nullptr;
  int rc = get_state(n, nullptr, &st);
  if (rc != TP_OK) return rc;
  return st->nnz;
}

int tp_words(int n, uint32_t *d_codes, hipStream_t stream) {
  TP_REQUIRE(n >= 1 && n <= 13, "n = %d outside 1..13", n);
  TP_REQUIRE(d_codes != nullptr, "d_codes is NULL");
  TP_HIP_CHECK(launch_words(n, d_codes, nullptr, nullptr, stream));
  return TP_OK;
}

int tp_build_state_matrix(int n, int dtype, void *d_A, int64_t lda, hipStream_t stream) {
  TP_REQUIRE(n >= 1 && n <= 13, "n = %d outside 1..13", n);
  TP_REQUIRE(valid_dtype(dtype), "bad dtype %d", dtype);
  const int64_t N = word_count_host(n);
  TP_REQUIRE(lda >= N, "lda = %lld < N = %lld", (long long)lda, (long long)N);
  TP_REQUIRE(d_A != nullptr, "d_A is NULL");
  std::lock_guard<std::mutex> lk(g_mu);
  State *st = nullptr;
  int rc = get_state(n, stream, &st);
  if (rc != TP_OK) return rc;
  TP_HIP_CHECK(launch_dense_state(n, N, (const uint32_t *)st->masks.ptr, dtype, d_A, lda, stream));
  return TP_OK;
}

int tp_build_state_csr(int n, int64_t *d_rowptr, uint32_t *d_col, uint8_t *d_z,
                       hipStream_t stream) {
  TP_REQUIRE(n >= 1 && n <= 13, "n = %d outside 1..13", n);
  TP_REQUIRE(d_rowptr != nullptr, "d_rowptr is NULL");
  std::lock_guard<std::mutex> lk(g_mu);
  State *st = nullptr;
  int rc = get_state(n, stream, &st);
  if (rc != TP_OK) return rc;
  const int64_t N = st->N;
  TP_HIP_CHECK(hipMemcpyAsync(d_rowptr, st->rowptr.ptr, (N + 1) * sizeof(int64_t),
                              hipMemcpyDeviceToDevice, stream));
  if (d_col && st->nnz > 0)
    TP_HIP_CHECK(hipMemcpyAsync(d_col, st->col.ptr, (size_t)st->nnz * sizeof(uint32_t),
                                hipMemcpyDeviceToDevice, stream));
  if (d_z) TP_HIP_CHECK(hipMemcpyAsync(d_z, st->z.ptr, N, hipMemcpyDeviceToDevice, stream));
  return TP_OK;
}

static int check_gemm(int dtype, int64_t M, int64_t N, int64_t K, const void *A, int64_t lda,
                      const void *B, int64_t ldb, const void *C, int64_t ldc) {
  TP_REQUIRE(valid_dtype(dtype), "bad dtype %d", dtype);
  TP_REQUIRE(M >= 0 && N >= 0 && K >= 0, "negative size");
  TP_REQUIRE(M < (1ll << 31) && N < (1ll << 31) && K < (1ll << 31), "size >= 2^31");
  TP_REQUIRE(lda >= (K > 0 ? K : 1) && ldb >= (N > 0 ? N : 1) && ldc >= (N > 0 ? N : 1),
             "leading dimension smaller than the row length");
  TP_REQUIRE((M == 0 || N == 0) || C != nullptr, "C is NULL");
  TP_REQUIRE((M == 0 || K == 0) || A != nullptr, "A is NULL");
  TP_REQUIRE((N == 0 || K == 0) || B != nullptr, "B is NULL");
  return TP_OK;
}

int tp_minplus_gemm(int dtype, int64_t M, int64_t N, int64_t K, const void *d_A, int64_t lda,
                    const void *d_B, int64_t ldb, void *d_C, int64_t ldc, int accumulate,
                    hipStream_t stream) {
  int rc = check_gemm(dtype, M, N, K, d_A, lda, d_B, ldb, d_C, ldc);
  if (rc != TP_OK) return rc;
  TP_HIP_CHECK(
      launch_gemm(dtype, M, N, K, d_A, lda, d_B, ldb, d_C, ldc, accumulate, -1, 0, stream));
  return TP_OK;
}

int tp_minplus_gemm_config(int dtype, int64_t M, int64_t N, int64_t K, const void *d_A,
                           int64_t lda, const void *d_B, int64_t ldb, void *d_C, int64_t ldc,
                           int accumulate, int config, hipStream_t stream) {
  int rc = check_gemm(dtype, M, N, K, d_A, lda, d_B, ldb, d_C, ldc);
  if (rc != TP_OK) return rc;
  TP_REQUIRE(config >= 0 && config < gemm_config_count(), "config %d outside 0..%d", config,
             gemm_config_count() - 1);
  TP_HIP_CHECK(launch_gemm(dtype, M, N, K, d_A, lda, d_B, ldb, d_C, ldc, accumulate, config, 1,
                           stream));
  return TP_OK;
}

int tp_minplus_gemm_ex(int dtype, int64_t M, int64_t N, int64_t K, const void *d_A, int64_t lda,
                       const void *d_B, int64_t ldb, void *d_C, int64_t ldc, int accumulate,
                       int config, int ksplit, hipStream_t stream) {
  int rc = check_gemm(dtype, M, N, K, d_A, lda, d_B, ldb, d_C, ldc);
  if (rc != TP_OK) return rc;
  TP_REQUIRE(config >= 0 && config < gemm_config_count(), "config %d outside 0..%d", config,
             gemm_config_count() - 1);
  TP_REQUIRE(ksplit >= 1 && ksplit <= 64, "ksplit %d outside 1..64", ksplit);
  TP_HIP_CHECK(launch_gemm(dtype, M, N, K, d_A, lda, d_B, ldb, d_C, ldc, accumulate, config,
                           ksplit, stream));
  return TP_OK;
}

int tp_minplus_gemm_ex_noalloc(int dtype, int64_t M, int64_t N, int64_t K, const void *d_A,
                               int64_t lda, const void *d_B, int64_t ldb, void *d_C,
                               int64_t ldc, int accumulate, int config, int ksplit,
                               hipStream_t stream) {
  int rc = check_gemm(dtype, M, N, K, d_A, lda, d_B, ldb, d_C, ldc);
  if (rc != TP_OK) return rc;
  TP_REQUIRE(config >= 0 && config < gemm_config_count(), "config %d outside 0..%d", config,
             gemm_config_count() - 1);
  TP_REQUIRE(ksplit >= 1 && ksplit <= 64, "ksplit %d outside 1..64", ksplit);
  return launch_gemm_fixed(dtype, M, N, K, d_A, lda, d_B, ldb, d_C, ldc, accumulate, config,
                           ksplit, stream);
}

int tp_gemm_config_count(void) { return gemm_config_count(); }

int tp_tune_planner(int n, double spmm_ops_per_s, double gemm_ops_per_s) {
  TP_REQUIRE(n >= 1 && n <= 12, "n = %d outside 1..12", n);
  const bool reset = spmm_ops_per_s == 0 && gemm_ops_per_s == 0;
  TP_REQUIRE(reset || (spmm_ops_per_s > 0 && gemm_ops_per_s > 0),
             "rates must be positive (or both 0)");
  std::lock_guard<std::mutex> lk(g_mu);
  g_spmm_rate[n] = reset ? kSpmmRate[n] : spmm_ops_per_s;
  g_gemm_rate[n] = reset ? kGemmRate[n] : gemm_ops_per_s;
  return TP_OK;
}

int tp_tune_gemm(int dtype, int64_t max_dim, int config, int ksplit) {
  TP_REQUIRE(valid_dtype(dtype), "bad dtype %d", dtype);
  if (max_dim >= 0) {
    TP_REQUIRE(config >= 0 && config < gemm_config_count(), "config %d outside 0..%d", config,
               gemm_config_count() - 1);
    TP_REQUIRE(ksplit >= 1 && ksplit <= 64, "ksplit %d outside 1..64", ksplit);
  }
  return gemm_tune_set(dtype, max_dim, config, ksplit);
}

int tp_gemm_choice(int dtype, int64_t M, int64_t N, int64_t K, int *config, int *ksplit) {
  TP_REQUIRE(valid_dtype(dtype), "bad dtype %d", dtype);
  TP_REQUIRE(M >= 0 && N >= 0 && K >= 0, "negative size");
  TP_REQUIRE(config != nullptr && ksplit != nullptr, "NULL output");
  gemm_choice(dtype, M, N, K, config, ksplit);
  return TP_OK;
}

int tp_minplus_gemv(int dtype, int64_t M, int64_t K, const void *d_A, int64_t lda,
                    const void *d_x, void *d_y, int trans, hipStream_t stream) {
  TP_REQUIRE(valid_dtype(dtype), "bad dtype %d", dtype);
  TP_REQUIRE(M >= 0 && K >= 0, "negative size");
  TP_REQUIRE(lda >= (K > 0 ? K : 1), "lda < K");
  TP_REQUIRE(trans == 0 || trans == 1, "trans must be 0 or 1");
  const int64_t ny = trans ? K : M;
  TP_REQUIRE(ny == 0 || d_y != nullptr, "y is NULL");
  TP_REQUIRE((M == 0 || K == 0) || (d_A != nullptr && d_x != nullptr), "A or x is NULL");
  if (!trans && K == 0 && M > 0) {
    // empty minimum: INF everywhere
    TP_HIP_CHECK(launch_fill_bytes(d_y, (size_t)M * elem_size(dtype), 0xFF, stream));
    return TP_OK;
  }
  if (trans && M == 0 && K > 0) {
    TP_HIP_CHECK(launch_fill_bytes(d_y, (size_t)K * elem_size(dtype), 0xFF, stream));
    return TP_OK;
  }
  TP_HIP_CHECK(launch_gemv(dtype, M, K, d_A, lda, d_x, d_y, trans, stream));
  return TP_OK;
}

int tp_minplus_spmm(int dtype, int64_t rows, int64_t K, const int64_t *d_rowptr,
                    const uint32_t *d_col, const uint8_t *d_z, const void *d_X, int64_t ldx,
                    void *d_Y, int64_t ldy, int64_t ncols, hipStream_t stream) {
  TP_REQUIRE(valid_dtype(dtype), "bad dtype %d", dtype);
  TP_REQUIRE(rows >= 0 && K >= 0 && ncols >= 0, "negative size");
  TP_REQUIRE(rows < (1ll << 31) && K < (1ll << 32), "size too large");
  TP_REQUIRE(ldx >= (ncols > 0 ? ncols : 1) && ldy >= (ncols > 0 ? ncols : 1),
             "leading dimension smaller than ncols");
  if (rows == 0 || ncols == 0) return TP_OK;
  TP_REQUIRE(d_rowptr && d_Y, "rowptr or Y is NULL");
  TP_REQUIRE(K == 0 || (d_col && d_z && d_X), "col, z or X is NULL");
  TP_HIP_CHECK(launch_spmm(dtype, rows, d_rowptr, d_col, d_z, d_X, ldx, d_Y, ldy, ncols, stream));
  return TP_OK;
}

int tp_trace_min(int dtype, int64_t N, const void *d_X, int64_t ldx, int32_t *d_out,
                 hipStream_t stream) {
  TP_REQUIRE(valid_dtype(dtype), "bad dtype %d", dtype);
  TP_REQUIRE(N >= 0 && ldx >= (N > 0 ? N : 1), "bad N or ldx");
  TP_REQUIRE(d_out != nullptr && (N == 0 || d_X != nullptr), "NULL pointer");
  TP_HIP_CHECK(launch_trace_min(dtype, N, d_X, ldx, d_out, stream));
  return TP_OK;
}

int tp_trace_of_product(int dtype, int64_t N, const void *d_X, int64_t ldx, const void *d_Y,
                        int64_t ldy, int32_t *d_out, hipStream_t stream) {
  TP_REQUIRE(valid_dtype(dtype), "bad dtype %d", dtype);
  TP_REQUIRE(N >= 0 && N < (1ll << 31), "bad N");
  TP_REQUIRE(ldx >= (N > 0 ? N : 1) && ldy >= (N > 0 ? N : 1), "leading dimension < N");
  TP_REQUIRE(d_out != nullptr && (N == 0 || (d_X && d_Y)), "NULL pointer");
  TP_HIP_CHECK(launch_trace_of_product(dtype, N, d_X, ldx, d_Y, ldy, d_out, stream));
  return TP_OK;
}

int tp_state_left_mul(int n, int form, const void *d_X, int64_t ldx, void *d_Y, int64_t ldy,
                      int64_t ncols, hipStream_t stream) {
  TP_REQUIRE(n >= 1 && n <= 13, "n = %d outside 1..13", n);
  TP_REQUIRE(form == TP_STEP_AUTO || form == TP_STEP_CSR || form == TP_STEP_BLOCKED ||
                 form == TP_STEP_BLOCKED_ENTRIES,
             "form %d is not TP_STEP_AUTO, TP_STEP_CSR, TP_STEP_BLOCKED or "
             "TP_STEP_BLOCKED_ENTRIES", form);
  TP_REQUIRE(ncols >= 0, "negative size");
  TP_REQUIRE(ldx >= (ncols > 0 ? ncols : 1) && ldy >= (ncols > 0 ? ncols : 1),
             "leading dimension < ncols");
  TP_REQUIRE(ncols == 0 || (d_X != nullptr && d_Y != nullptr), "X or Y is NULL");
  std::lock_guard<std::mutex> lk(g_mu);
  State *st = nullptr;
  const int rc = get_state(n, stream, &st);
  if (rc != TP_OK) return rc;
  TP_HIP_CHECK(state_step(st, form, (const uint16_t *)d_X, ldx, (uint16_t *)d_Y, ldy, ncols,
                          stream));
  return TP_OK;
}

int tp_tune_step(int n, int form) {
  TP_REQUIRE(n >= 1 && n <= 12, "n = %d outside 1..12", n);
  TP_REQUIRE(form == TP_STEP_AUTO || form == TP_STEP_CSR || form == TP_STEP_BLOCKED ||
                 form == TP_STEP_BLOCKED_ENTRIES,
             "form %d is not TP_STEP_AUTO, TP_STEP_CSR, TP_STEP_BLOCKED or "
             "TP_STEP_BLOCKED_ENTRIES", form);
  std::lock_guard<std::mutex> lk(g_mu);
  g_step_form[n] = form;
  return TP_OK;
}

int tp_sparse_trace_of_product(int dtype, int64_t N, const int64_t *d_rowptr,
                               const uint32_t *d_col, const uint8_t *d_z, const void *d_X,
                               int64_t ldx, int32_t *d_out, hipStream_t stream) {
  TP_REQUIRE(valid_dtype(dtype), "bad dtype %d", dtype);
  TP_REQUIRE(N >= 0 && ldx >= (N > 0 ? N : 1), "bad N or ldx");
  TP_REQUIRE(d_out != nullptr, "out is NULL");
  TP_REQUIRE(N == 0 || (d_rowptr && d_col && d_z && d_X), "NULL pointer");
  TP_HIP_CHECK(launch_fill_i32(d_out, 1, dtype == TP_U16 ? 0xFFFF : 0xFF, stream));
  TP_HIP_CHECK(launch_sparse_trace(dtype, N, d_rowptr, d_col, d_z, d_X, ldx, d_out, stream));
  return TP_OK;
}

int tp_tropical_power_trace(int n, int64_t m, int32_t *gamma2_host, hipStream_t stream) {
  TP_REQUIRE(n >= 1 && n <= 12, "n = %d outside 1..12", n);
  TP_REQUIRE(m >= 3, "the cycle order m = %lld must be at least 3", (long long)m);
  TP_REQUIRE(gamma2_host != nullptr, "gamma2_host is NULL");
  if ((int64_t)n * m >= 0xFFFF) {
    set_error("n * m = %lld could reach INF = 65535 in 16-bit entries", (long long)(n * m));
    return TP_EOVERFLOW;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  return power_trace_locked(n, m, gamma2_host, stream);
}

int64_t tp_state_select(int n, int max_zeros, int32_t *d_idx, int64_t cap, hipStream_t stream) {
  TP_REQUIRE(n >= 1 && n <= 13, "n = %d outside 1..13", n);
  TP_REQUIRE(max_zeros >= 0, "negative zero count");
  std::lock_guard<std::mutex> lk(g_mu);
  State *st = nullptr;
  int rc = get_state(n, stream, &st);
  if (rc != TP_OK) return rc;
  const int32_t *idx = nullptr;
  int64_t cnt = 0;
  rc = state_selection(st, std::min(max_zeros, n), stream, &idx, &cnt);
  if (rc != TP_OK) return rc;
  if (d_idx != nullptr) {
    TP_REQUIRE(cap >= cnt, "%lld states selected, room for %lld", (long long)cnt,
               (long long)cap);
    if (cnt > 0)
      TP_HIP_CHECK(hipMemcpyAsync(d_idx, idx, (size_t)cnt * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, stream));
  }
  return cnt;
}

int tp_build_state_columns(int n, const int32_t *d_idx, int64_t count, void *d_X, int64_t ldx,
                           hipStream_t stream) {
  TP_REQUIRE(n >= 1 && n <= 13, "n = %d outside 1..13", n);
  TP_REQUIRE(count >= 0 && count < ((int64_t)1 << 31), "count out of range");
  TP_REQUIRE(count == 0 || (d_idx != nullptr && d_X != nullptr), "NULL pointer");
  TP_REQUIRE(ldx >= count, "leading dimension below count");
  std::lock_guard<std::mutex> lk(g_mu);
  State *st = nullptr;
  int rc = get_state(n, stream, &st);
  if (rc != TP_OK) return rc;
  TP_HIP_CHECK(launch_state_columns(n, st->N, (const uint32_t *)st->masks.ptr, d_idx, count,
                                    (uint16_t *)d_X, ldx, stream));
  return TP_OK;
}

int tp_diag_select_min(int64_t N, int64_t count, const int32_t *d_idx, const void *d_X,
                       int64_t ldx, int32_t *d_out, hipStream_t stream) {
  TP_REQUIRE(N >= 0 && count >= 0, "negative size");
  TP_REQUIRE(d_out != nullptr, "d_out is NULL");
  TP_REQUIRE(count == 0 || (d_idx != nullptr && d_X != nullptr), "NULL pointer");
  TP_REQUIRE(ldx >= count, "leading dimension below count");
  TP_HIP_CHECK(launch_diag_select_min(N, count, d_idx, (const uint16_t *)d_X, ldx, d_out, stream));
  return TP_OK;
}

int tp_tune_prune(int mode) {
  TP_REQUIRE(mode >= -1 && mode <= 1, "mode is -1, 0 or 1");
  std::lock_guard<std::mutex> lk(g_mu);
  g_prune = mode;
  return TP_OK;
}

int tp_release_cache(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto &kv : g_states) {
    release(kv.second.masks);
    release(kv.second.z);
    release(kv.second.rowptr);
    release(kv.second.col);
    release(kv.second.colz);
    release(kv.second.bptr);
    release(kv.second.bent);
    release(kv.second.order);
    release(kv.second.border);
    release(kv.second.fptr);
    release(kv.second.fent);
    release(kv.second.finfo);
    release(kv.second.forder);
    for (auto &sb : kv.second.sel) release(sb.second);
  }
  g_states.clear();
  for (auto &kv : g_ws) {
    for (auto &b : kv.second.buf) release(b);
    release(kv.second.scalar);
  }
  g_ws.clear();
  cyclic_release_cache();
  return TP_OK;
}

}  // extern "C"
