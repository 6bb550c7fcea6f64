// C ABI of the small-cycle / any-path walk (cyclic.hip): argument checks, the
// per-device cache of cyclic column digraphs, the plain walk by (min,+)
// vector-matrix products and the sweep of every path order up to a bound.
//
// gamma_2(P_n x C_m) = min_p (start x A^(n-1))_p + end_p, with A the column
// digraph of the cyclic words of length m (Section 2.1's construction with
// Section 2.2's rules read around the cycle; Section 1 names the problem).
// Each product is exact on integers, so every form below gives the same
// numbers: the dense vector-matrix product (tp_minplus_gemv's kernel, the
// companion work's form), a gather-min over predecessor lists per level, or
// the whole walk inside one workgroup.
#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace tp {

namespace {

struct Buf {
  void *ptr = nullptr;
  size_t bytes = 0;
};

hipError_t grow(Buf &b, size_t bytes) {
  if (b.ptr && b.bytes >= bytes) return hipSuccess;
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

void drop(Buf &b) {
  if (b.ptr) (void)hipFree(b.ptr);
  b = Buf{};
}

// Per (device, m): masks, zero counts, predecessor CSR, the walk's order of
// columns (longest predecessor list first), the one-workgroup strips, the
// boundary vectors (u16), a dense u16 copy of A for the vector-matrix form,
// and two level vectors plus scalars of workspace.
struct Cyc {
  int m = 0;
  int64_t N = 0, nnz = -1, ld = 0;
  Buf masks, z, predptr, pred, order, strips, start, end, dense, vec[2], scalar;
  Buf items, ym;  // the step form's work items and 32-bit level minima
  int64_t nitems = 0;
  bool dense_ready = false;
};

std::mutex g_cmu;
std::map<std::pair<int, int>, Cyc> g_cyc;

int device_now() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}

// Largest N whose walk runs inside one workgroup (x in 16 bits and the
// gathered minima in 32 bits, in 64 KB of LDS with room for the reduction).
constexpr int64_t kChainMaxN = (65536 - 1024) / 6;
// Arcs up to which the one-workgroup walk beats two launches per level
// (measured per level: m = 7, 21,080 arcs: 4.1 against 5.4 us; m = 8, 86,855
// arcs: 13.5 against 5.5 us).
constexpr int64_t kChainMaxNnz = 1 << 15;

int get_cyc(int m, hipStream_t s, Cyc **out) {
  Cyc &c = g_cyc[{device_now(), m}];
  if (c.nnz < 0) {
    c.m = m;
    c.N = cyclic_count_host(m);
    const int64_t N = c.N;
    c.ld = (N + 63) / 64 * 64;
    TP_HIP_CHECK(grow(c.masks, N * sizeof(uint32_t)));
    TP_HIP_CHECK(grow(c.z, N));
    TP_HIP_CHECK(grow(c.predptr, (N + 1) * sizeof(int64_t)));
    TP_HIP_CHECK(grow(c.start, N * sizeof(uint16_t)));
    TP_HIP_CHECK(grow(c.end, N * sizeof(uint16_t)));
    TP_HIP_CHECK(grow(c.vec[0], N * sizeof(uint16_t)));
    TP_HIP_CHECK(grow(c.vec[1], N * sizeof(uint16_t)));
    TP_HIP_CHECK(grow(c.scalar, 64));
    TP_HIP_CHECK(launch_cyclic_words(m, nullptr, (uint8_t *)c.z.ptr, (uint32_t *)c.masks.ptr, s));
    TP_HIP_CHECK(launch_cyclic_boundary(m, N, (const uint32_t *)c.masks.ptr, TP_U16, c.start.ptr,
                                        c.end.ptr, s));
    TP_HIP_CHECK(launch_cyclic_pred_count(m, N, (const uint32_t *)c.masks.ptr,
                                          (int64_t *)c.predptr.ptr, s));
    TP_HIP_CHECK(launch_scan_rowptr(N, (int64_t *)c.predptr.ptr, s));
    std::vector<int64_t> pp((size_t)N + 1);
    TP_HIP_CHECK(hipMemcpyAsync(pp.data(), c.predptr.ptr, pp.size() * sizeof(int64_t),
                                hipMemcpyDeviceToHost, s));
    TP_HIP_CHECK(hipStreamSynchronize(s));
    const int64_t nnz = pp[(size_t)N];
    TP_HIP_CHECK(grow(c.pred, (size_t)std::max<int64_t>(nnz, 1) * sizeof(uint16_t)));
    TP_HIP_CHECK(launch_cyclic_pred_fill(m, N, (const uint32_t *)c.masks.ptr,
                                         (const int64_t *)c.predptr.ptr, (uint16_t *)c.pred.ptr,
                                         s));
    std::vector<int32_t> ord((size_t)N);
    for (int64_t i = 0; i < N; ++i) ord[(size_t)i] = (int32_t)i;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
      return pp[a + 1] - pp[a] > pp[b + 1] - pp[b];
    });
    TP_HIP_CHECK(grow(c.order, N * sizeof(int32_t)));
    TP_HIP_CHECK(hipMemcpyAsync(c.order.ptr, ord.data(), ord.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, s));
    std::vector<char> items;
    c.nitems = cyclic_items_host(N, pp.data(), ord.data(), &items);
    TP_HIP_CHECK(grow(c.items, std::max<size_t>(items.size(), 16)));
    if (!items.empty())
      TP_HIP_CHECK(hipMemcpyAsync(c.items.ptr, items.data(), items.size(), hipMemcpyHostToDevice,
                                  s));
    TP_HIP_CHECK(grow(c.ym, N * sizeof(uint32_t)));
    if (N <= kChainMaxN) {
      const int64_t per = cyclic_strip_length(nnz);
      TP_HIP_CHECK(grow(c.strips, (size_t)per * 1024 * sizeof(uint32_t)));
      TP_HIP_CHECK(launch_cyclic_strips(N, nnz, (const int64_t *)c.predptr.ptr,
                                        (const uint16_t *)c.pred.ptr, (uint32_t *)c.strips.ptr, s));
    }
    TP_HIP_CHECK(hipStreamSynchronize(s));
    c.nnz = nnz;
  }
  *out = &c;
  return TP_OK;
}

int get_dense(Cyc *c, hipStream_t s) {
  if (!c->dense_ready) {
    TP_HIP_CHECK(grow(c->dense, (size_t)c->N * (size_t)c->ld * sizeof(uint16_t)));
    TP_HIP_CHECK(launch_cyclic_dense(c->m, c->N, (const uint32_t *)c->masks.ptr, TP_U16,
                                     c->dense.ptr, c->ld, s));
    c->dense_ready = true;
  }
  return TP_OK;
}

bool valid_m(int m) { return m >= 3 && m <= 12; }

// Levels 2..nmax by `form` after the answer of level 1 is in out[0]; x holds
// level 1 (start) on entry.  out[k - 1] must hold INF for the step form.
int walk_levels(Cyc *c, int64_t nmax, int form, int32_t *out, hipStream_t s) {
  const int64_t N = c->N;
  uint16_t *x = (uint16_t *)c->vec[0].ptr, *y = (uint16_t *)c->vec[1].ptr;
  for (int64_t k = 2; k <= nmax; ++k) {
    if (form == TP_WALK_GEMV) {
      TP_HIP_CHECK(launch_gemv(TP_U16, N, N, c->dense.ptr, c->ld, x, y, 1, s));
      TP_HIP_CHECK(launch_cyclic_answer(N, y, (const uint16_t *)c->end.ptr, out + (k - 1), s));
    } else {
      TP_HIP_CHECK(launch_cyclic_step(N, c->nitems, c->items.ptr, (const uint16_t *)c->pred.ptr,
                                      (const uint8_t *)c->z.ptr, (const uint16_t *)c->end.ptr,
                                      (uint32_t *)c->ym.ptr, x, y, out + (k - 1), s));
    }
    std::swap(x, y);
  }
  return TP_OK;
}

int pick_form(const Cyc *c, int form) {
  if (form != TP_WALK_AUTO) return form;
  return (c->N <= kChainMaxN && c->nnz <= kChainMaxNnz) ? TP_WALK_CHAIN : TP_WALK_STEPS;
}

}  // namespace

void cyclic_release_cache() {
  std::lock_guard<std::mutex> lk(g_cmu);
  for (auto &kv : g_cyc) {
    Cyc &c = kv.second;
    for (Buf *b : {&c.masks, &c.z, &c.predptr, &c.pred, &c.order, &c.strips, &c.start, &c.end,
                   &c.dense, &c.vec[0], &c.vec[1], &c.scalar, &c.items, &c.ym})
      drop(*b);
  }
  g_cyc.clear();
}

}  // namespace tp

using namespace tp;

extern "C" {

int64_t tp_cyclic_dim(int m) {
  if (!valid_m(m)) {
    set_error("m = %d outside 3..12", m);
    return TP_EINVAL;
  }
  return cyclic_count_host(m);
}

int64_t tp_cyclic_nnz(int m) {
  if (!valid_m(m)) {
    set_error("m = %d outside 3..12", m);
    return TP_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_cmu);
  Cyc *c = nullptr;
  const int rc = get_cyc(m, nullptr, &c);
  if (rc != TP_OK) return rc;
  return c->nnz;
}

int tp_cyclic_words(int m, uint32_t *d_codes, hipStream_t stream) {
  TP_REQUIRE(valid_m(m), "m = %d outside 3..12", m);
  TP_REQUIRE(d_codes != nullptr, "d_codes is NULL");
  TP_HIP_CHECK(launch_cyclic_words(m, d_codes, nullptr, nullptr, stream));
  return TP_OK;
}

int tp_build_cyclic_matrix(int m, int dtype, void *d_A, int64_t lda, hipStream_t stream) {
  TP_REQUIRE(valid_m(m), "m = %d outside 3..12", m);
  TP_REQUIRE(dtype == TP_U8 || dtype == TP_U16, "bad dtype %d", dtype);
  const int64_t N = cyclic_count_host(m);
  TP_REQUIRE(lda >= N, "lda = %lld < N = %lld", (long long)lda, (long long)N);
  TP_REQUIRE(d_A != nullptr, "d_A is NULL");
  std::lock_guard<std::mutex> lk(g_cmu);
  Cyc *c = nullptr;
  const int rc = get_cyc(m, stream, &c);
  if (rc != TP_OK) return rc;
  TP_HIP_CHECK(launch_cyclic_dense(m, N, (const uint32_t *)c->masks.ptr, dtype, d_A, lda, stream));
  return TP_OK;
}

int tp_build_cyclic_boundary(int m, int dtype, void *d_start, void *d_end, hipStream_t stream) {
  TP_REQUIRE(valid_m(m), "m = %d outside 3..12", m);
  TP_REQUIRE(dtype == TP_U8 || dtype == TP_U16, "bad dtype %d", dtype);
  TP_REQUIRE(d_start != nullptr || d_end != nullptr, "both vectors are NULL");
  std::lock_guard<std::mutex> lk(g_cmu);
  Cyc *c = nullptr;
  const int rc = get_cyc(m, stream, &c);
  if (rc != TP_OK) return rc;
  TP_HIP_CHECK(launch_cyclic_boundary(m, c->N, (const uint32_t *)c->masks.ptr, dtype, d_start,
                                      d_end, stream));
  return TP_OK;
}

int tp_cyclic_walk_gamma2(int64_t n, int m, int32_t *gamma2_host, hipStream_t stream) {
  TP_REQUIRE(valid_m(m), "m = %d outside 3..12", m);
  TP_REQUIRE(n >= 1, "the path order n = %lld must be at least 1", (long long)n);
  TP_REQUIRE(gamma2_host != nullptr, "gamma2_host is NULL");
  if (n * (int64_t)m >= 0xFFFF) {
    set_error("n * m = %lld could reach INF = 65535 in 16-bit entries", (long long)(n * m));
    return TP_EOVERFLOW;
  }
  std::lock_guard<std::mutex> lk(g_cmu);
  Cyc *c = nullptr;
  int rc = get_cyc(m, stream, &c);
  if (rc != TP_OK) return rc;
  rc = get_dense(c, stream);
  if (rc != TP_OK) return rc;
  int32_t *d_out = (int32_t *)c->scalar.ptr;
  uint16_t *x = (uint16_t *)c->vec[0].ptr, *y = (uint16_t *)c->vec[1].ptr;
  TP_HIP_CHECK(hipMemcpyAsync(x, c->start.ptr, (size_t)c->N * sizeof(uint16_t),
                              hipMemcpyDeviceToDevice, stream));
  for (int64_t k = 2; k <= n; ++k) {
    TP_HIP_CHECK(launch_gemv(TP_U16, c->N, c->N, c->dense.ptr, c->ld, x, y, 1, stream));
    std::swap(x, y);
  }
  TP_HIP_CHECK(launch_cyclic_answer(c->N, x, (const uint16_t *)c->end.ptr, d_out, stream));
  int32_t host = 0;
  TP_HIP_CHECK(hipMemcpyAsync(&host, d_out, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  TP_HIP_CHECK(hipStreamSynchronize(stream));
  *gamma2_host = host;
  return TP_OK;
}

int tp_cyclic_walk_sweep(int m, int64_t nmax, int32_t *d_gamma2, int form, hipStream_t stream) {
  TP_REQUIRE(valid_m(m), "m = %d outside 3..12", m);
  TP_REQUIRE(nmax >= 1, "nmax = %lld must be at least 1", (long long)nmax);
  TP_REQUIRE(d_gamma2 != nullptr, "d_gamma2 is NULL");
  TP_REQUIRE(form >= TP_WALK_AUTO && form <= TP_WALK_GEMV, "bad form %d", form);
  if (nmax * (int64_t)m >= 0xFFFF) {
    set_error("nmax * m = %lld could reach INF = 65535 in 16-bit entries",
              (long long)(nmax * m));
    return TP_EOVERFLOW;
  }
  std::lock_guard<std::mutex> lk(g_cmu);
  Cyc *c = nullptr;
  int rc = get_cyc(m, stream, &c);
  if (rc != TP_OK) return rc;
  const int f = pick_form(c, form);
  if (f == TP_WALK_CHAIN) {
    TP_REQUIRE(c->N <= kChainMaxN, "m = %d: %lld words do not fit one workgroup's LDS", m,
               (long long)c->N);
    TP_HIP_CHECK(launch_cyclic_chain(c->N, c->nnz, nmax, (const uint32_t *)c->strips.ptr,
                                     (const uint8_t *)c->z.ptr, (const uint16_t *)c->start.ptr,
                                     (const uint16_t *)c->end.ptr, d_gamma2, stream));
    return TP_OK;
  }
  if (f == TP_WALK_GEMV) {
    rc = get_dense(c, stream);
    if (rc != TP_OK) return rc;
  }
  TP_HIP_CHECK(launch_fill_i32(d_gamma2, nmax, 0xFFFF, stream));
  if (f == TP_WALK_STEPS)
    TP_HIP_CHECK(launch_fill_u32((uint32_t *)c->ym.ptr, c->N, 0xFFFFu, stream));
  TP_HIP_CHECK(hipMemcpyAsync(c->vec[0].ptr, c->start.ptr, (size_t)c->N * sizeof(uint16_t),
                              hipMemcpyDeviceToDevice, stream));
  TP_HIP_CHECK(launch_cyclic_answer(c->N, (const uint16_t *)c->vec[0].ptr,
                                    (const uint16_t *)c->end.ptr, d_gamma2, stream));
  rc = walk_levels(c, nmax, f, d_gamma2, stream);
  if (rc != TP_OK) return rc;
  // the level vectors are the cache's own: wait before another call may use them
  TP_HIP_CHECK(hipStreamSynchronize(stream));
  return TP_OK;
}

}  // extern "C"
