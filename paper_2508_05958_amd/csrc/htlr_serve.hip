// Request server: continuous batching of solve requests (see include/htlr.h).
//
// Work is scheduled per unit: the structures of one group key (structures
// that share their factors) or one structure alone.  A unit is idle or has
// one step in flight.  Every tick:
//   1. admission: queued requests enter first come first served while the
//      device bytes of resident structures plus request state fit the budget
//      (idle structures are evicted least recently used first);
//   2. for each idle unit with active requests, on its streams: one fused
//      FP64 product for the requests that need their refinement residual, and
//      one fused inner-precision product for the requests in a GMRES cycle,
//      followed by their per-request Arnoldi updates (classical Gram-Schmidt
//      twice, on the device); an event marks the end of the step;
//   3. the host waits until at least one unit in flight has finished its
//      step, then makes the host-side Givens updates and state transitions of
//      the finished units' requests;
//   4. finished requests are retired; their buffers go to a pool for the
//      next admissions (freeing device memory would wait for the device).
// So a unit advances at its own pace: small structures take many steps
// while a large one computes one product.
// Fused products gather the requests' vectors into a column-major batch and
// call the HTLR product with nrhs = batch width; with use_graphs the gather
// and the product are replayed from a hipGraph captured per (precision,
// width).

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <set>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "htlr_handle.h"
#include "htlr_vec.h"

namespace htlr {

extern thread_local std::string g_last_error;
htlr_status record(const Error& e);

namespace {

#define HTLR_CHECK_ST(call)                                \
  do {                                                     \
    htlr_status s_ = (call);                               \
    if (s_ != HTLR_OK) ::htlr::fail(s_, g_last_error);     \
  } while (0)

struct PinnedBuf {
  double* p = nullptr;
  size_t n = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  PinnedBuf(PinnedBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  PinnedBuf& operator=(PinnedBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  void alloc(size_t count) {
    release();
    HTLR_HIP(hipHostMalloc((void**)&p, count * sizeof(double), hipHostMallocDefault));
    n = count;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
  }
  ~PinnedBuf() { release(); }
};

struct Structure;

struct Req {
  int64_t id = 0;
  std::string key;
  Structure* S = nullptr;
  // copied request parameters
  std::vector<double> f, a, points;
  int kernel = 0, d = 0, n = 0, p = 0, leaf = 0, adm = 0;
  double eta2 = 1.0, tol = 1e-8;
  int max_outer = 50;
  int64_t N = 0;
  // lifecycle
  int state = 0, status = HTLR_OK;
  double t_submit = 0, t_admit = -1, t_done = -1;
  std::vector<double> result;
  // device state: f | x | r | d | V[0..m]
  DevBuf dev;
  size_t dev_bytes = 0;
  double *df = nullptr, *dx = nullptr, *dr = nullptr, *dd = nullptr, *V = nullptr;
  DevBuf hdev;             // device scalars: h pass 1 [m+1], h pass 2 [m+1], norm, y [m]
  PinnedBuf host;          // pinned mirror of hdev
  bool ready = false;      // f and x = 0 written to the device (done when its unit is idle)
  // GMRES-IR state
  double fn = 0, rn = 0, beta = 0, rtol = 0;
  int outer = 0, inner = 0, k = 0;
  bool arnoldi = false;
  std::vector<double> H, cs, sn, g, y;
};

struct Structure {
  std::string key;
  std::string gkey;                // structures with equal gkey share their factors
  std::vector<double> points, a;   // build inputs, compared on a key hit
  hipEvent_t ev = nullptr;         // orders a group's work after this structure's stream
  hipEvent_t done = nullptr;       // end of the structure's step in flight
  htlr_matrix A = nullptr;
  int64_t N = 0;
  int inner = HTLR_FP32;           // precision of its inner products (bfloat16 cores need a uniform grid)
  size_t bytes = 0;
  int active = 0;
  double last_use = 0;
  hipStream_t stream = nullptr;
  int cap = 0;
  DevBuf U64, F64, U32, F32, ptrs, partial;
  PinnedBuf hptrs;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;
  std::map<std::pair<int, int>, int> uses;
  size_t ptr_slot = 0;     // next free slot of hptrs in this tick (uploads are asynchronous)
  ~Structure() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    if (A) htlr_free(A);
    if (ev) (void)hipEventDestroy(ev);
    if (done) (void)hipEventDestroy(done);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

// Batch buffers of the fused products of a group of structures that share
// their factors (uniform grids of the same d, n, p, leaf, eta2 and
// admissibility; the kernel and a(x) may differ): the products of all their
// requests in one tick run as one grouped product (product_group), whose up
// contractions and down expansions cover every member's columns in one
// launch per level.
// A grouped product replayed from a captured hipGraph: one per composition
// (members, their column counts, precision, tick slot).  The column tables
// of that composition live in its own pinned and device buffers, which the
// captured copy reads on every replay.
struct GroupGraph {
  hipGraphExec_t exec = nullptr;
  PinnedBuf ht;
  DevBuf td;
  int grouped = 0;                 // grouped launches per replay
  ~GroupGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

constexpr size_t kMaxGroupGraphs = 64;   // captured compositions kept per group

struct Group {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;       // end of the group's step in flight
  int cols = 0;                    // columns of the batch buffers
  DevBuf U64, F64, U32, F32, ptrs, partial, tabs;
  PinnedBuf hptrs, htabs;
  size_t bytes = 0;
  std::map<std::string, std::unique_ptr<GroupGraph>> graphs;
  std::map<std::string, int> uses;
  // graphs hold the addresses of the batch buffers and of the members' work
  // buffers: dropped when either may change
  void drop_graphs() {
    if (stream) (void)hipStreamSynchronize(stream);
    graphs.clear();
    uses.clear();
  }
  ~Group() {
    if (stream) (void)hipStreamSynchronize(stream);
    graphs.clear();
    if (done) (void)hipEventDestroy(done);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

constexpr int kTabSlots = 2 * kMaxLevels;   // column tables per grouped product

constexpr int kRedB = 512;

}  // namespace

struct ServerImpl {
  htlr_server_opts o{};
  size_t budget = 0, used = 0;
  // relative residual an inner GMRES cycle aims at, per inner precision:
  // bfloat16-core products are within about 1e-5 of FP64 on these grids (the
  // near field and the factors stay FP32), so a cycle can aim at 1e-4 and
  // two refinement steps reach 1e-8 (1e-2 took four, each with an FP64 product)
  double inner_tol_for(int prec) const {
    if (o.inner_tol > 0) return o.inner_tol;
    return prec == HTLR_FP32 ? 1e-6 : (prec == HTLR_BF16_CORE ? 1e-4 : 1e-12);
  }
  int64_t next_id = 1;
  std::deque<int64_t> queue;
  std::map<int64_t, std::unique_ptr<Req>> reqs;
  std::map<std::string, std::unique_ptr<Structure>> structs;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  htlr_server_stats_t st{};

  // The step of one unit (the structures of a group key) on the device: the
  // requests it advances and the events (one per stream used) that end it.
  struct Flight {
    std::vector<Req*> reqs;
    std::vector<hipEvent_t> evs;
  };
  std::map<std::string, Flight> flights;   // by group key

  // Buffers of retired requests, reused by later admissions: freeing device
  // or pinned memory would wait for all work on the device.  The device
  // bytes of dev_pool stay counted in used until the pool is released.
  std::multimap<size_t, DevBuf> dev_pool;
  std::vector<DevBuf> hdev_pool;
  std::vector<PinnedBuf> host_pool;
  size_t pooled = 0;

  void release_pool() {
    used -= pooled;
    pooled = 0;
    dev_pool.clear();
    hdev_pool.clear();
    host_pool.clear();
  }

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // Structure key: the build arguments, eta2 by its exact bit pattern, and a
  // hash of the points and a(x); a hit is confirmed by comparing points and
  // a in full (same_inputs), so a hash collision never reuses a structure.
  static std::string make_key(const Req& q) {
    std::ostringstream os;
    uint64_t eb;
    std::memcpy(&eb, &q.eta2, 8);
    os << q.kernel << '|' << q.d << '|' << q.n << '|' << q.p << '|' << q.leaf << '|' << std::hex << eb << std::dec
       << '|' << q.adm << '|';
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const std::vector<double>& v) {
      for (double x : v) {
        uint64_t b;
        std::memcpy(&b, &x, 8);
        h = (h ^ b) * 1099511628211ull;
      }
      h = (h ^ v.size()) * 1099511628211ull;
    };
    mix(q.points);
    mix(q.a);
    os << h;
    return os.str();
  }

  size_t state_bytes(int64_t N) const { return ((size_t)(o.restart + 5) * N * sizeof(double) + 4095) & ~size_t(4095); }

  // device bytes a new structure will hold: the matrix plus product work
  // buffers and the fused batch buffers for cap columns
  size_t structure_bytes(const Req& q) const {
    htlr_build_opts bo{};
    bo.eta2 = q.eta2;
    bo.admissibility = q.adm;
    size_t fp = 0;
    HTLR_CHECK_ST(htlr_footprint(q.points.empty() ? nullptr : q.points.data(), (htlr_kernel)q.kernel, q.d, q.n, q.p,
                                 q.leaf, &bo, &fp));
    int L = 0;
    std::vector<int> m;
    tree_shape(q.d, q.n, q.leaf, &L, &m);
    size_t P = 1, ws = 0;
    for (int l = 0; l < q.d; ++l) P *= q.p;
    for (int l = 0; l <= L; ++l) {
      size_t nb = 1;
      for (int k = 0; k < q.d; ++k) nb *= (size_t)(q.n / m[l]);
      if (l >= 2) ws += nb * (size_t)o.max_batch * P * 16;
    }
    return fp + ws + (size_t)q.N * o.max_batch * 24 + (size_t)kRedB * (o.restart + 2) * 8;
  }

  void evict_idle(size_t need) {
    while (used + need > budget) {
      Structure* victim = nullptr;
      for (auto& kv : structs)
        if (kv.second->active == 0 && (!victim || kv.second->last_use < victim->last_use)) victim = kv.second.get();
      if (!victim) return;
      used -= victim->bytes;
      auto g = groups.find(victim->gkey);
      if (g != groups.end()) g->second->drop_graphs();
      structs.erase(victim->key);
      ++st.evictions;
    }
  }

  static bool same_inputs(const Structure& S, const Req& q) { return S.points == q.points && S.a == q.a; }

  // Structures on the uniform cell-centred grid with the same (d, n, p,
  // leaf, eta2, admissibility) have the same cluster and block trees and the
  // same factors at every level; only the kernel (cores, near field) and
  // a(x) differ.  Other structures form groups of one.
  static std::string group_key(const Req& q) {
    if (!q.points.empty()) return "solo|" + q.key;
    uint64_t eb;
    std::memcpy(&eb, &q.eta2, 8);
    std::ostringstream os;
    os << "uniform|" << q.d << '|' << q.n << '|' << q.p << '|' << q.leaf << '|' << std::hex << eb << std::dec << '|'
       << q.adm;
    return os.str();
  }

  std::map<std::string, std::unique_ptr<Group>> groups;

  Structure* build(Req& q) {
    auto S = std::make_unique<Structure>();
    S->key = q.key;
    S->N = q.N;
    S->points = q.points;
    S->a = q.a;
    S->gkey = group_key(q);
    htlr_build_opts bo{};
    bo.eta2 = q.eta2;
    bo.admissibility = q.adm;
    bo.a = q.a.empty() ? nullptr : q.a.data();
    bo.precisions = (1 << HTLR_FP64) | (1 << o.inner_prec);
    // bfloat16 cores exist on uniform grids only: given points may form a
    // tensor grid, whose inner products then run in FP32
    const bool maybe_tensor = o.inner_prec == HTLR_BF16_CORE && !q.points.empty();
    if (maybe_tensor) bo.precisions |= 1 << HTLR_FP32;
    HTLR_CHECK_ST(htlr_build(q.points.empty() ? nullptr : q.points.data(), (htlr_kernel)q.kernel, q.d, q.n, q.p,
                             q.leaf, &bo, &S->A));
    S->inner = (maybe_tensor && !S->A->uniform) ? HTLR_FP32 : o.inner_prec;
    HTLR_HIP(hipStreamCreate(&S->stream));
    HTLR_HIP(hipEventCreateWithFlags(&S->ev, hipEventDisableTiming));
    HTLR_HIP(hipEventCreateWithFlags(&S->done, hipEventDisableTiming));
    S->cap = o.max_batch;
    S->U64.alloc((size_t)S->N * S->cap * sizeof(double));
    S->F64.alloc((size_t)S->N * S->cap * sizeof(double));
    if (S->inner != HTLR_FP64) {
      S->U32.alloc((size_t)S->N * S->cap * sizeof(float));
      S->F32.alloc((size_t)S->N * S->cap * sizeof(float));
    }
    S->ptrs.alloc((size_t)S->cap * sizeof(double*));
    // one slot of cap pointers per fused product of a tick
    S->hptrs.alloc((size_t)S->cap * (2 * ((o.max_active + S->cap - 1) / S->cap) + 2));
    S->partial.alloc((size_t)kRedB * (o.restart + 2) * sizeof(double));
    if (o.autotune) {
      // tune the fused product shapes this structure will see
      for (int w = 1; w <= S->cap; w *= 2) {
        HTLR_CHECK_ST(htlr_autotune(S->A, w, HTLR_FP64, nullptr));
        if (S->inner != HTLR_FP64) HTLR_CHECK_ST(htlr_autotune(S->A, w, (htlr_precision)S->inner, nullptr));
      }
    }
    {
      std::lock_guard<std::mutex> lk(S->A->ws_mu);
      reserve_workspace(*S->A, S->cap);
    }
    htlr_info_t inf{};
    HTLR_CHECK_ST(htlr_info(S->A, &inf));
    size_t wsb = 0;
    HTLR_CHECK_ST(htlr_workspace_bytes(S->A, S->cap, HTLR_FP64, &wsb));
    S->bytes = inf.device_bytes + wsb + S->A->ws.extra_bytes() + S->U64.bytes + S->F64.bytes + S->U32.bytes + S->F32.bytes + S->partial.bytes;
    Structure* raw = S.get();
    structs[q.key] = std::move(S);
    ++st.structures_built;
    return raw;
  }

  void admit() {
    int active = 0;
    for (auto& kv : reqs)
      if (kv.second->state == 1) ++active;
    while (!queue.empty() && active < o.max_active) {
      Req& q = *reqs.at(queue.front());
      auto it = structs.find(q.key);
      // a key whose structure was built for other points or a(x) (a hash
      // collision) is made distinct until it names a free or matching slot
      while (it != structs.end() && !same_inputs(*it->second, q)) {
        q.key += '#';
        it = structs.find(q.key);
      }
      Structure* S = it == structs.end() ? nullptr : it->second.get();
      const size_t sb = state_bytes(q.N);
      auto pit = dev_pool.find(sb);
      size_t need = (pit != dev_pool.end() ? 0 : sb) + (S ? 0 : structure_bytes(q));
      if (used + need > budget && pooled) {
        release_pool();
        pit = dev_pool.end();
        need = sb + (S ? 0 : structure_bytes(q));
      }
      if (used + need > budget) evict_idle(need);
      if (used + need > budget) {
        if (active == 0 && structs.empty() && !S) {
          // the estimate is an upper bound; decide on the built size
          S = build(q);
          if (S->bytes + sb > budget) {
            structs.erase(q.key);
            q.state = 3;
            q.status = HTLR_ERR_OOM;
            q.t_done = now();
            queue.pop_front();
            continue;
          }
          used += S->bytes;
        } else {
          break;
        }
      } else if (!S) {
        S = build(q);
        used += S->bytes;
      }
      q.S = S;
      if (pit != dev_pool.end()) {
        q.dev = std::move(pit->second);
        dev_pool.erase(pit);
        pooled -= sb;
      } else {
        q.dev.alloc(sb);
        used += sb;
      }
      q.dev_bytes = sb;
      double* base = q.dev.as<double>();
      q.df = base;
      q.dx = base + q.N;
      q.dr = base + 2 * q.N;
      q.dd = base + 3 * q.N;
      q.V = base + 4 * q.N;
      const int m = o.restart;
      if (!hdev_pool.empty()) {
        q.hdev = std::move(hdev_pool.back());
        hdev_pool.pop_back();
      } else {
        q.hdev.alloc((size_t)(3 * m + 4) * sizeof(double));
      }
      if (!host_pool.empty()) {
        q.host = std::move(host_pool.back());
        host_pool.pop_back();
      } else {
        q.host.alloc((size_t)(3 * m + 4));
      }
      q.ready = false;   // f and x = 0 go to the device when the unit is next idle
      q.H.assign((size_t)(m + 1) * m, 0.0);
      q.cs.assign(m, 0.0);
      q.sn.assign(m, 0.0);
      q.g.assign(m + 1, 0.0);
      q.y.assign(m, 0.0);
      q.fn = -1.0;   // ||f|| computed with the first residual
      q.arnoldi = false;
      q.state = 1;
      q.t_admit = now();
      ++S->active;
      S->last_use = q.t_admit;
      ++active;
      queue.pop_front();
    }
  }

  // fused product of columns src[0..c) into out (F64 or F32) on S's stream
  void fused_product(Structure* S, int prec, const std::vector<const double*>& src) {
    const int c = (int)src.size();
    static_assert(sizeof(const double*) == sizeof(double), "pointer table packs pointers into 8-byte slots");
    if (S->ptr_slot + S->cap > S->hptrs.n) fail(HTLR_ERR_INVALID, "too many fused products in one tick");
    const double** hp = reinterpret_cast<const double**>(S->hptrs.p + S->ptr_slot);
    S->ptr_slot += S->cap;
    for (int j = 0; j < c; ++j) hp[j] = src[j];
    HTLR_HIP(hipMemcpyAsync(S->ptrs.ptr, hp, c * sizeof(double*), hipMemcpyHostToDevice, S->stream));
    auto launch = [&]() {
      const int nb = vblocks(S->N);
      if (prec == HTLR_FP64) {
        hipLaunchKernelGGL(k_gather_f64, dim3(nb), dim3(256), 0, S->stream, S->ptrs.as<const double*>(),
                           S->U64.as<double>(), S->N, c);
        HTLR_CHECK_ST(htlr_matvec(S->A, S->U64.ptr, S->F64.ptr, c, HTLR_FP64, HTLR_VEC_F64, S->stream));
      } else {
        hipLaunchKernelGGL(k_gather_f32, dim3(nb), dim3(256), 0, S->stream, S->ptrs.as<const double*>(),
                           S->U32.as<float>(), S->N, c);
        HTLR_CHECK_ST(htlr_matvec(S->A, S->U32.ptr, S->F32.ptr, c, (htlr_precision)prec, HTLR_VEC_F32, S->stream));
      }
    };
    const auto key = std::make_pair(prec, c);
    ++st.fused_products;
    if (!o.use_graphs) {
      launch();
      return;
    }
    auto g = S->graphs.find(key);
    if (g != S->graphs.end()) {
      HTLR_HIP(hipGraphLaunch(g->second, S->stream));
      ++st.graph_launches;
      return;
    }
    if (S->uses[key]++ == 0) {   // first use runs eagerly: work buffers and work lists get allocated
      launch();
      return;
    }
    hipGraph_t graph = nullptr;
    HTLR_HIP(hipStreamBeginCapture(S->stream, hipStreamCaptureModeRelaxed));
    try {
      launch();
    } catch (...) {
      (void)hipStreamEndCapture(S->stream, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    HTLR_HIP(hipStreamEndCapture(S->stream, &graph));
    hipGraphExec_t exec = nullptr;
    HTLR_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    S->graphs[key] = exec;
    HTLR_HIP(hipGraphLaunch(exec, S->stream));
    ++st.graph_launches;
  }

  // device: out[c] = <Vb[:, c], x> into dst (device), c < ncols, on stream st
  // with the partial-sum buffer part (kRedB x ncols doubles)
  void dots(hipStream_t st, double* part, int64_t N, const double* Vb, int ncols, const double* x, double* dst) {
    hipLaunchKernelGGL(k_dots_partial, dim3(kRedB), dim3(kRB), 0, st, Vb, N, ncols, x, N, part);
    hipLaunchKernelGGL(k_dots_final, dim3(ncols), dim3(kRB), 0, st, part, kRedB, ncols, dst);
  }

  // refinement residual r = f - A x from column col of an FP64 product (col
  // null: x = 0, the request's first residual, r = f), its norm (and ||f||
  // the first time) copied to the host
  void post_residual(Req* q, const double* col, hipStream_t st, double* part) {
    const int m = o.restart;
    const int64_t N = q->N;
    if (col)
      hipLaunchKernelGGL(k_sub_to, dim3(vblocks(N)), dim3(256), 0, st, q->df, col, q->dr, N);
    else
      HTLR_HIP(hipMemcpyAsync(q->dr, q->df, N * sizeof(double), hipMemcpyDeviceToDevice, st));
    double* hd = q->hdev.as<double>();
    dots(st, part, N, q->dr, 1, q->dr, hd + 2 * (m + 1));
    if (q->fn < 0) dots(st, part, N, q->df, 1, q->df, hd + 2 * (m + 1) + 1);
    HTLR_HIP(hipMemcpyAsync(q->host.p, hd, (3 * m + 4) * sizeof(double), hipMemcpyDeviceToHost, st));
  }

  // The first residual of a request (x = 0) needs no product: r = f.
  static bool first_residual(const Req& q) { return !q.arnoldi && q.fn < 0; }

  // Arnoldi step: w = A V_k from column col64 (FP64 product) or col32 (inner
  // precision product), classical Gram-Schmidt twice, norm to the host
  void post_arnoldi(Req* q, const double* col64, const float* col32, hipStream_t st, double* part) {
    const int m = o.restart;
    const int64_t N = q->N;
    double* w = q->V + (int64_t)(q->k + 1) * N;
    if (col64)
      HTLR_HIP(hipMemcpyAsync(w, col64, N * sizeof(double), hipMemcpyDeviceToDevice, st));
    else
      hipLaunchKernelGGL(k_f2d, dim3(vblocks(N)), dim3(256), 0, st, col32, w, N);
    double* hd = q->hdev.as<double>();
    for (int pass = 0; pass < 2; ++pass) {
      double* hp = hd + pass * (m + 1);
      dots(st, part, N, q->V, q->k + 1, w, hp);
      hipLaunchKernelGGL(k_sub_vh, dim3(vblocks(N)), dim3(256), 0, st, q->V, N, q->k + 1, hp, w, N);
    }
    dots(st, part, N, w, 1, w, hd + 2 * (m + 1));
    HTLR_HIP(hipMemcpyAsync(q->host.p, hd, (3 * m + 4) * sizeof(double), hipMemcpyDeviceToHost, st));
  }

  // A request's f and x = 0 on the device, on its structure's stream (its
  // unit is idle, so the copy does not wait behind a step in flight).
  void init_req(Req* q) {
    if (q->ready) return;
    HTLR_HIP(hipMemcpyAsync(q->df, q->f.data(), q->N * sizeof(double), hipMemcpyHostToDevice, q->S->stream));
    hipLaunchKernelGGL(k_zero, dim3(vblocks(q->N)), dim3(256), 0, q->S->stream, q->dx, q->N);
    q->ready = true;
  }

  void issue(Structure* S, std::vector<Req*>& members) {
    const int64_t N = S->N;
    double* part = S->partial.as<double>();
    for (Req* q : members) init_req(q);
    std::vector<Req*> R, K;
    for (Req* q : members) {
      if (q->arnoldi) K.push_back(q);
      else if (first_residual(*q)) post_residual(q, nullptr, S->stream, part);
      else R.push_back(q);
    }
    // refinement residuals: r = f - A x (FP64)
    for (size_t s = 0; s < R.size(); s += o.max_batch) {
      const size_t e = std::min(R.size(), s + (size_t)o.max_batch);
      std::vector<const double*> src;
      for (size_t i = s; i < e; ++i) src.push_back(R[i]->dx);
      fused_product(S, HTLR_FP64, src);
      for (size_t i = s; i < e; ++i)
        post_residual(R[i], S->F64.as<double>() + (int64_t)(i - s) * N, S->stream, part);
    }
    // Arnoldi steps: w = A V_k (inner precision), CGS2, norm
    const int ip = S->inner;
    for (size_t s = 0; s < K.size(); s += o.max_batch) {
      const size_t e = std::min(K.size(), s + (size_t)o.max_batch);
      std::vector<const double*> src;
      for (size_t i = s; i < e; ++i) src.push_back(K[i]->V + (int64_t)K[i]->k * N);
      fused_product(S, ip, src);
      for (size_t i = s; i < e; ++i) {
        if (ip == HTLR_FP64)
          post_arnoldi(K[i], S->F64.as<double>() + (int64_t)(i - s) * N, nullptr, S->stream, part);
        else
          post_arnoldi(K[i], nullptr, S->F32.as<float>() + (int64_t)(i - s) * N, S->stream, part);
      }
    }
    HTLR_HIP(hipGetLastError());
  }

  // The group of structures Ss (same gkey, each with active requests) ready
  // for one grouped product per precision this tick, or null when they do not
  // fit one (a structure with more than max_batch requests in one phase, more
  // than kMaxGroupCols columns, or no memory for the batch buffers).
  Group* group_for(const std::string& gk, const std::vector<Structure*>& Ss,
                   std::map<Structure*, std::vector<Req*>>& by) {
    int nr = 0, nk = 0;
    for (Structure* S : Ss) {
      int r = 0, k = 0;
      for (Req* q : by[S])
        if (q->arnoldi) ++k;
        else if (!first_residual(*q)) ++r;
      if (r > o.max_batch || k > o.max_batch) return nullptr;
      nr += r;
      nk += k;
    }
    const int need = std::max(nr, nk);
    if (need > kMaxGroupCols) return nullptr;
    auto& slot = groups[gk];
    if (!slot) {
      slot = std::make_unique<Group>();
      HTLR_HIP(hipStreamCreate(&slot->stream));
      HTLR_HIP(hipEventCreateWithFlags(&slot->done, hipEventDisableTiming));
      slot->ptrs.alloc((size_t)2 * kMaxGroupCols * sizeof(double*));
      slot->hptrs.alloc((size_t)2 * kMaxGroupCols);
      slot->partial.alloc((size_t)kRedB * (o.restart + 2) * sizeof(double));
      slot->tabs.alloc((size_t)2 * kTabSlots * sizeof(ColTab));
      slot->htabs.alloc((size_t)2 * kTabSlots * sizeof(ColTab) / sizeof(double));
      // (plus the column tables of up to kMaxGroupGraphs captured compositions)
      slot->bytes = slot->ptrs.bytes + slot->partial.bytes + slot->tabs.bytes +
                    kMaxGroupGraphs * (size_t)kTabSlots * sizeof(ColTab);
      used += slot->bytes;
    }
    Group* G = slot.get();
    if (G->cols < need) {
      const int64_t N = Ss[0]->N;
      const int cols = std::min(kMaxGroupCols, std::max(need, 2 * o.max_batch));
      const bool f32 = Ss[0]->inner != HTLR_FP64;
      const size_t per = (size_t)N * cols * (sizeof(double) * 2 + (f32 ? sizeof(float) * 2 : 0));
      const size_t old = (size_t)N * G->cols * (sizeof(double) * 2 + (f32 ? sizeof(float) * 2 : 0));
      if (used - old + per > budget) return nullptr;
      G->drop_graphs();
      G->U64.alloc((size_t)N * cols * sizeof(double));
      G->F64.alloc((size_t)N * cols * sizeof(double));
      if (f32) {
        G->U32.alloc((size_t)N * cols * sizeof(float));
        G->F32.alloc((size_t)N * cols * sizeof(float));
      }
      used = used - old + per;
      G->bytes += per - old;
      G->cols = cols;
    }
    return G;
  }

  // One grouped product of the given precision over the requests in Q (in
  // structure order), reading column src[i] of request Q[i].
  void group_product(Group* G, int prec, int slot, const std::vector<Structure*>& Ss,
                     const std::vector<int>& cols, const std::vector<const double*>& src) {
    const int C = (int)src.size();
    const int64_t N = Ss[0]->N;
    const double** hp = reinterpret_cast<const double**>(G->hptrs.p) + (size_t)slot * kMaxGroupCols;
    for (int j = 0; j < C; ++j) hp[j] = src[j];
    const double** dp = G->ptrs.as<const double*>() + (size_t)slot * kMaxGroupCols;
    HTLR_HIP(hipMemcpyAsync(dp, hp, C * sizeof(double*), hipMemcpyHostToDevice, G->stream));
    std::vector<htlr_matrix_impl*> As;
    for (Structure* S : Ss) As.push_back(S->A);
    // gather + grouped product with the given column-table buffers
    auto launch = [&](ColTab* th, ColTab* td) -> int {
      if (prec == HTLR_FP64) {
        hipLaunchKernelGGL(k_gather_f64, dim3(vblocks(N)), dim3(256), 0, G->stream, dp, G->U64.as<double>(), N, C);
        return product_group(As, cols, G->U64.ptr, G->F64.ptr, prec, G->stream, th, td);
      }
      hipLaunchKernelGGL(k_gather_f32, dim3(vblocks(N)), dim3(256), 0, G->stream, dp, G->U32.as<float>(), N, C);
      return product_group(As, cols, G->U32.ptr, G->F32.ptr, prec, G->stream, th, td);
    };
    ++st.fused_products;
    ++st.group_products;
    if (o.use_graphs) {
      std::ostringstream ks;
      ks << prec << '|' << slot;
      for (size_t i = 0; i < Ss.size(); ++i) ks << '|' << (const void*)Ss[i] << ':' << cols[i];
      const std::string key = ks.str();
      auto it = G->graphs.find(key);
      if (it != G->graphs.end()) {
        HTLR_HIP(hipGraphLaunch(it->second->exec, G->stream));
        st.grouped_launches += it->second->grouped;
        ++st.graph_launches;
        return;
      }
      // first use runs eagerly (work lists and buffers exist afterwards);
      // a composition seen again is captured with its own column tables
      if (G->uses[key]++ > 0 && G->graphs.size() < kMaxGroupGraphs) {
        auto g = std::make_unique<GroupGraph>();
        g->ht.alloc((size_t)kTabSlots * sizeof(ColTab) / sizeof(double));
        g->td.alloc((size_t)kTabSlots * sizeof(ColTab));
        hipGraph_t graph = nullptr;
        HTLR_HIP(hipStreamBeginCapture(G->stream, hipStreamCaptureModeRelaxed));
        try {
          g->grouped = launch(reinterpret_cast<ColTab*>(g->ht.p), g->td.as<ColTab>());
        } catch (...) {
          (void)hipStreamEndCapture(G->stream, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          throw;
        }
        HTLR_HIP(hipStreamEndCapture(G->stream, &graph));
        const hipError_t ie = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HTLR_HIP(ie);
        HTLR_HIP(hipGraphLaunch(g->exec, G->stream));
        st.grouped_launches += g->grouped;
        ++st.graph_launches;
        G->graphs[key] = std::move(g);
        return;
      }
    }
    st.grouped_launches += launch(reinterpret_cast<ColTab*>(G->htabs.p) + (size_t)slot * kTabSlots,
                                  G->tabs.as<ColTab>() + (size_t)slot * kTabSlots);
  }

  void issue_group(Group* G, const std::vector<Structure*>& Ss, std::map<Structure*, std::vector<Req*>>& by) {
    for (Structure* S : Ss)
      for (Req* q : by[S]) init_req(q);
    // after each member's earlier work (refinement updates issued on its stream)
    for (Structure* S : Ss) {
      HTLR_HIP(hipEventRecord(S->ev, S->stream));
      HTLR_HIP(hipStreamWaitEvent(G->stream, S->ev, 0));
    }
    const int64_t N = Ss[0]->N;
    double* part = G->partial.as<double>();
    for (Structure* S : Ss)
      for (Req* q : by[S])
        if (first_residual(*q)) post_residual(q, nullptr, G->stream, part);
    for (int phase = 0; phase < 2; ++phase) {
      // phase 0: refinement residuals (FP64); phase 1: Arnoldi steps (inner precision)
      std::vector<Structure*> mem;
      std::vector<int> cols;
      std::vector<Req*> Q;
      std::vector<const double*> src;
      for (Structure* S : Ss) {
        int c = 0;
        for (Req* q : by[S])
          if (q->arnoldi == (phase == 1) && !first_residual(*q)) {
            Q.push_back(q);
            src.push_back(phase == 0 ? q->dx : q->V + (int64_t)q->k * N);
            ++c;
          }
        if (c) {
          mem.push_back(S);
          cols.push_back(c);
        }
      }
      if (Q.empty()) continue;
      const int prec = phase == 0 ? HTLR_FP64 : Ss[0]->inner;   // members of a group share their grid
      group_product(G, prec, phase, mem, cols, src);
      for (size_t i = 0; i < Q.size(); ++i) {
        if (phase == 0)
          post_residual(Q[i], G->F64.as<double>() + (int64_t)i * N, G->stream, part);
        else if (prec == HTLR_FP64)
          post_arnoldi(Q[i], G->F64.as<double>() + (int64_t)i * N, nullptr, G->stream, part);
        else
          post_arnoldi(Q[i], nullptr, G->F32.as<float>() + (int64_t)i * N, G->stream, part);
      }
    }
    HTLR_HIP(hipGetLastError());
  }

  void finish_one(Req& q) {
    Structure* S = q.S;
    const int m = o.restart;
    const int64_t N = S->N;
    const double* hh = q.host.p;
    if (!q.arnoldi) {
      if (q.fn < 0) q.fn = std::sqrt(hh[2 * (m + 1) + 1]);
      q.rn = std::sqrt(hh[2 * (m + 1)]);
      if (!std::isfinite(q.rn) || !std::isfinite(q.fn)) {
        q.state = 3;
        q.status = HTLR_ERR_NUMERIC;
        return;
      }
      if (q.fn == 0.0 || q.rn <= q.tol * q.fn) {
        q.state = 2;
        q.status = HTLR_OK;
        return;
      }
      if (q.outer >= q.max_outer) {
        q.state = 3;
        q.status = HTLR_ERR_NOT_CONVERGED;
        return;
      }
      // start a GMRES cycle on A d = r
      ++q.outer;
      q.beta = q.rn;
      q.rtol = std::max(inner_tol_for(q.S->inner), q.tol * q.fn / q.rn);
      hipLaunchKernelGGL(k_scale_to, dim3(vblocks(N)), dim3(256), 0, S->stream, q.dr, 1.0 / q.beta, q.V, N);
      std::fill(q.g.begin(), q.g.end(), 0.0);
      q.g[0] = q.beta;
      q.k = 0;
      q.arnoldi = true;
      return;
    }
    const int k = q.k;
    std::vector<double> h(k + 2);
    for (int j = 0; j <= k; ++j) h[j] = hh[j] + hh[(m + 1) + j];
    const double hn = std::sqrt(hh[2 * (m + 1)]);
    if (!std::isfinite(hn)) {
      q.state = 3;
      q.status = HTLR_ERR_NUMERIC;
      return;
    }
    h[k + 1] = hn;
    double* w = q.V + (int64_t)(k + 1) * N;
    if (hn > 0) hipLaunchKernelGGL(k_scale_to, dim3(vblocks(N)), dim3(256), 0, S->stream, w, 1.0 / hn, w, N);
    for (int j = 0; j < k; ++j) {
      const double t = q.cs[j] * h[j] + q.sn[j] * h[j + 1];
      h[j + 1] = -q.sn[j] * h[j] + q.cs[j] * h[j + 1];
      h[j] = t;
    }
    const double den = std::hypot(h[k], h[k + 1]);
    q.cs[k] = den > 0 ? h[k] / den : 1.0;
    q.sn[k] = den > 0 ? h[k + 1] / den : 0.0;
    h[k] = den;
    q.g[k + 1] = -q.sn[k] * q.g[k];
    q.g[k] = q.cs[k] * q.g[k];
    for (int j = 0; j <= k; ++j) q.H[(size_t)j * m + k] = h[j];
    ++q.inner;
    q.k = k + 1;
    const bool conv = std::fabs(q.g[k + 1]) <= q.rtol * q.beta || hn == 0.0;
    if (conv || q.k == m) {
      // x += V y with y = R^{-1} g; the next tick recomputes the FP64 residual
      const int kk = q.k;
      for (int i = kk - 1; i >= 0; --i) {
        double s = q.g[i];
        for (int j = i + 1; j < kk; ++j) s -= q.H[(size_t)i * m + j] * q.y[j];
        q.y[i] = s / q.H[(size_t)i * m + i];
      }
      double* yd = q.hdev.as<double>() + 2 * (m + 1) + 2;
      std::memcpy(q.host.p + 2 * (m + 1) + 2, q.y.data(), kk * sizeof(double));
      HTLR_HIP(hipMemcpyAsync(yd, q.host.p + 2 * (m + 1) + 2, kk * sizeof(double), hipMemcpyHostToDevice, S->stream));
      hipLaunchKernelGGL(k_add_vy, dim3(vblocks(N)), dim3(256), 0, S->stream, q.V, N, kk, yd, q.dx, N);
      q.arnoldi = false;
    }
  }

  void retire(Req& q) {
    Structure* S = q.S;
    q.result.resize(q.N);
    // on the structure's own stream: a copy on the null stream would wait
    // for every unit in flight
    HTLR_HIP(hipMemcpyAsync(q.result.data(), q.dx, q.N * sizeof(double), hipMemcpyDeviceToHost, S->stream));
    HTLR_HIP(hipStreamSynchronize(S->stream));
    q.t_done = now();
    dev_pool.emplace(q.dev_bytes, std::move(q.dev));
    pooled += q.dev_bytes;
    if ((int)hdev_pool.size() < o.max_active) hdev_pool.push_back(std::move(q.hdev));
    if ((int)host_pool.size() < o.max_active) host_pool.push_back(std::move(q.host));
    q.hdev.release();
    q.host.release();
    --S->active;
    S->last_use = q.t_done;
    q.S = nullptr;
  }

  void step(int* active, int* queued) {
    ++st.ticks;
    admit();
    // requests of idle units
    std::map<Structure*, std::vector<Req*>> by;
    for (auto& kv : reqs) {
      Req* q = kv.second.get();
      if (q->state == 1 && !flights.count(q->S->gkey)) by[q->S].push_back(q);
    }
    std::map<std::string, std::vector<Structure*>> bygroup;
    for (auto& g : by) bygroup[g.first->gkey].push_back(g.first);
    for (auto& kv : bygroup) {
      Flight fl;
      Group* G = (!o.no_group_fusion && kv.second.size() >= 2) ? group_for(kv.first, kv.second, by) : nullptr;
      if (G) {
        issue_group(G, kv.second, by);
        HTLR_HIP(hipEventRecord(G->done, G->stream));
        fl.evs.push_back(G->done);
      } else {
        for (Structure* S : kv.second) {
          S->ptr_slot = 0;   // the unit is idle: its earlier pointer uploads are done
          issue(S, by[S]);
          HTLR_HIP(hipEventRecord(S->done, S->stream));
          fl.evs.push_back(S->done);
        }
      }
      for (Structure* S : kv.second)
        for (Req* q : by[S]) fl.reqs.push_back(q);
      flights[kv.first] = std::move(fl);
    }
    // wait until at least one unit has finished its step
    std::vector<std::string> ready;
    while (!flights.empty()) {
      for (auto& kv : flights) {
        bool done = true;
        for (hipEvent_t e : kv.second.evs) {
          const hipError_t r = hipEventQuery(e);
          if (r == hipErrorNotReady) {
            done = false;
            break;
          }
          HTLR_HIP(r);
        }
        if (done) ready.push_back(kv.first);
      }
      if (!ready.empty()) break;
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    for (const std::string& k : ready) {
      Flight fl = std::move(flights[k]);
      flights.erase(k);
      for (Req* q : fl.reqs) {
        finish_one(*q);
        if (q->state >= 2) retire(*q);
      }
    }
    // batch buffers of groups with fewer than two resident structures go
    // (not while a step of the group is in flight)
    for (auto it = groups.begin(); it != groups.end();) {
      int resident = 0;
      for (auto& kv : structs)
        if (kv.second->gkey == it->first) ++resident;
      if (resident < 2 && !flights.count(it->first)) {
        used -= it->second->bytes;
        it = groups.erase(it);
      } else {
        ++it;
      }
    }
    int a = 0;
    for (auto& kv : reqs)
      if (kv.second->state == 1) ++a;
    if (active) *active = a;
    if (queued) *queued = (int)queue.size();
  }
};

}  // namespace htlr

struct htlr_server_s : htlr::ServerImpl {};

using namespace htlr;

extern "C" {

htlr_status htlr_server_create(const htlr_server_opts* opts, htlr_server* out) {
  if (!out) { g_last_error = "out is NULL"; return HTLR_ERR_INVALID; }
  *out = nullptr;
  try {
    auto S = std::make_unique<htlr_server_s>();
    if (opts) S->o = *opts;
    if (S->o.max_active <= 0) S->o.max_active = 64;
    if (S->o.max_batch <= 0) S->o.max_batch = 16;
    if (S->o.max_batch > 64) fail(HTLR_ERR_INVALID, "max_batch must be <= 64");
    if (S->o.restart <= 0) S->o.restart = 30;
    if (S->o.restart > 200) fail(HTLR_ERR_INVALID, "restart too large");
    const int ip = S->o.inner_prec;
    if (ip != HTLR_FP64 && ip != HTLR_FP32 && ip != HTLR_BF16_CORE) fail(HTLR_ERR_INVALID, "unknown inner precision");
    S->budget = S->o.memory_budget;
    if (!S->budget) {
      size_t fr = 0, tot = 0;
      HTLR_HIP(hipMemGetInfo(&fr, &tot));
      S->budget = (size_t)(0.9 * (double)fr);
    }
    *out = S.release();
    return HTLR_OK;
  } catch (const Error& e) {
    return record(e);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HTLR_ERR_INVALID;
  }
}

htlr_status htlr_server_submit(htlr_server S, const htlr_request* r, int64_t* id) {
  if (!S || !r || !id || !r->f) { g_last_error = "null argument"; return HTLR_ERR_INVALID; }
  try {
    auto q = std::make_unique<Req>();
    q->kernel = r->kernel;
    q->d = r->d;
    q->n = r->n;
    q->p = r->p;
    q->leaf = r->leaf;
    q->adm = r->admissibility;
    q->eta2 = r->eta2 > 0 ? r->eta2 : 1.0;
    q->tol = r->tol > 0 ? r->tol : 1e-8;
    q->max_outer = r->max_outer > 0 ? r->max_outer : 50;
    if (q->d != 2 && q->d != 3) fail(HTLR_ERR_UNSUPPORTED, "d must be 2 or 3");
    if (q->n < 1) fail(HTLR_ERR_INVALID, "n must be positive");
    q->N = 1;
    for (int l = 0; l < q->d; ++l) q->N *= q->n;
    q->f.assign(r->f, r->f + q->N);
    if (r->a) q->a.assign(r->a, r->a + q->N);
    if (r->points) q->points.assign(r->points, r->points + (size_t)q->d * q->n);
    q->key = ServerImpl::make_key(*q);
    q->id = S->next_id++;
    q->t_submit = S->now();
    *id = q->id;
    S->queue.push_back(q->id);
    S->reqs[q->id] = std::move(q);
    return HTLR_OK;
  } catch (const Error& e) {
    return record(e);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HTLR_ERR_INVALID;
  }
}

htlr_status htlr_server_step(htlr_server S, int* active, int* queued) {
  if (!S) { g_last_error = "null server"; return HTLR_ERR_INVALID; }
  try {
    S->step(active, queued);
    return HTLR_OK;
  } catch (const Error& e) {
    return record(e);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HTLR_ERR_INVALID;
  }
}

htlr_status htlr_server_result(htlr_server S, int64_t id, double* u, htlr_request_info* info) {
  if (!S) { g_last_error = "null server"; return HTLR_ERR_INVALID; }
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) { g_last_error = "unknown request id"; return HTLR_ERR_INVALID; }
  Req& q = *it->second;
  if (info) {
    info->state = q.state;
    info->status = q.status;
    info->outer_iters = q.outer;
    info->inner_iters = q.inner;
    info->rel_residual = q.fn > 0 ? q.rn / q.fn : 0.0;
    info->t_submit = q.t_submit;
    info->t_admit = q.t_admit;
    info->t_done = q.t_done;
  }
  if (q.state < 2) { g_last_error = "request not finished"; return HTLR_ERR_INVALID; }
  if (u && !q.result.empty()) std::memcpy(u, q.result.data(), q.N * sizeof(double));
  S->reqs.erase(it);
  return HTLR_OK;
}

htlr_status htlr_server_stats(htlr_server S, htlr_server_stats_t* out) {
  if (!S || !out) { g_last_error = "null argument"; return HTLR_ERR_INVALID; }
  *out = S->st;
  out->resident_structures = (int)S->structs.size();
  out->resident_bytes = S->used;
  int a = 0;
  for (auto& kv : S->reqs)
    if (kv.second->state == 1) ++a;
  out->active = a;
  out->queued = (int)S->queue.size();
  return HTLR_OK;
}

double htlr_server_clock(htlr_server S) { return S ? S->now() : 0.0; }

void htlr_server_destroy(htlr_server S) {
  if (!S) return;
  (void)hipDeviceSynchronize();
  delete S;
}

}  // extern "C"
