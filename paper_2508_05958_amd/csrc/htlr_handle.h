// The HTLR matrix handle: everything htlr_build leaves resident in HBM, plus
// the work buffers of products.  Shared by construction, product and solver.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "htlr_internal.h"

namespace htlr {

#define HTLR_HIP(call)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      ::htlr::fail(e_ == hipErrorOutOfMemory ? HTLR_ERR_OOM : HTLR_ERR_HIP,               \
                   std::string(#call) + ": " + hipGetErrorString(e_));                   \
  } while (0)

// Device allocation owned by a handle.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : ptr(o.ptr), bytes(o.bytes) { o.ptr = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); ptr = o.ptr; bytes = o.bytes; o.ptr = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t b) {
    release();
    if (b == 0) return;
    HTLR_HIP(hipMalloc(&ptr, b));
    bytes = b;
  }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(ptr); }
};

// One level of the cluster tree that carries admissible leaves.
struct LevelData {
  int level = 0, B = 0, m = 0;
  int rank = 0, P = 0;               // Tucker rank of the level's factors and cores (P = rank^d)
  int64_t nbox = 0, npairs = 0;
  DevBuf ptr, src, cid;              // CSR of admissible leaves; core id per entry (uniform)
  const Csr* csr = nullptr;          // pair lists of the matrix-core work lists (nullptr: the
                                     // plan's admissible leaves of this level)
  DevBuf U64, V64, U32, V32;         // factors: uniform [m][p]; tensor [d][B][m][p]
  DevBuf cheb64, cheb32;             // tensor grids: Chebyshev points [d][B][p]
  int ncore = 0;                     // uniform grids: one core per offset
  std::vector<int> offsets;          // 3 ints per core: sigma - tau in boxes
  DevBuf Gm16, Gm32, Gm64;           // cores, layout [core][t][s] (s fastest)
  // matrix-core kernel work lists, per number of boxes per tile (uniform grids)
  struct Tiles {
    int nb = 0;
    int64_t ntile = 0;
    DevBuf tau;                      // [ntile][nb] target boxes (-1 = empty slot)
    DevBuf ptr;                      // [ntile + 1] into off
    DevBuf off;                      // int4 (core id, offset x, y, z) per entry
    std::vector<int64_t> class_start;  // first tile of each parity class
    std::vector<int64_t> len;          // offset-list length of each tile (host)
    int64_t maxlist = 0;             // longest offset list of a tile
    struct Items {
      DevBuf buf;                    // work items (tile << 12 | row block << 6 | split)
      int n = 0;
    };
    std::map<int, Items> items;      // per number of K splits
  };
  std::vector<Tiles> tiles;
  // offset-major work lists (one GEMM per offset; outputs per pair, then reduced)
  struct OffsetTiles {
    int nb = 0, nmb = 0;
    int64_t npairs = 0;
    int nitems = 0;
    DevBuf tau, out, ptr, off, items;  // tiles as in Tiles, plus output slots
    DevBuf rptr;                       // per box: first slot of its pairs (consecutive, offset order)
  };
  std::vector<OffsetTiles> otiles;
};

struct Workspace {
  int nrhs = 0;
  bool frozen = false;               // reserved: products must not reallocate
  std::vector<DevBuf> W, H, W16;     // per level
  std::vector<DevBuf> UP;            // per level: partial up contractions of split boxes
  DevBuf zero;                       // a zero source tensor (matrix-core kernel)
  // per level (levels run concurrently): K-split partial sums of the
  // matrix-core kernel, per-pair products of the offset-major mode
  std::vector<DevBuf> parts, pairs;
  DevBuf nparts;                     // K-split partial sums (leaf-column near field)
  size_t bytes = 0;                  // W, H, UP and zero
  size_t extra_bytes() const {
    size_t b = nparts.bytes;
    for (const DevBuf& x : parts) b += x.bytes;
    for (const DevBuf& x : pairs) b += x.bytes;
    return b;
  }
};

// hipEvent pairs around product launches, for measurement.
struct Profiler {
  bool on = false;
  struct Rec { std::string name; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    HTLR_HIP(hipEventCreate(&e));
    return e;
  }
  void clear() {
    for (auto& r : recs) { pool.push_back(r.a); pool.push_back(r.b); }
    recs.clear();
  }
  ~Profiler() {
    clear();
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// Kernel variant choices for products of one shape (nrhs, precision).
struct TuneParams {
  int ks_target = 0;                 // matrix-core core apply: workgroups aimed for when splitting K
                                     // (0 automatic: at least 2048, and 4 per unsplit work item)
  int near_kind = -1;                // -1 automatic, 0 VALU row kernel, 1 matrix-core kernel with
                                     // right-hand sides as columns, 2 with target leaves as columns,
                                     // 3 the generic uniform-grid kernel (no row reuse)
                                     // 4 the near field as class tiles of the matrix-core core
                                     // apply (one 512 x 512 block per near offset)
  int near_nw = 0;                   // VALU row kernel: waves per leaf (0 automatic)
  int near_ks = 0;                   // leaf-column near kernel: K splits (0 automatic)
  int near_tpw = 0;                  // leaf-column near kernel: 16-row tiles per wave, 4 or 8 (0 = 8)
  int near_ct = 0;                   // leaf-column near kernel: 16-column tiles per wave, 1 or 2 (0 = 1)
  int tile = 0;                      // matrix-core tile: 0 automatic, 1 128x128, 2 128x64, 3 256x128,
                                     // 4 224x64 (FP64), 5 256x256 (BF16), 6 64x128, 7 64x64
  int core_mode = 0;                 // 0 automatic, 1 class tiles, 2 offset-major
  int serial = 0;                    // level launches: 1 every launch on the caller's stream, 2 levels on
                                     // side streams, concurrently; 0 automatic (levels_serial)
  int order = -1;                    // matrix-core work items: 0 (class, row block, split, tile),
                                     // 1 (class, tile, row block, split): the row blocks of a tile
                                     // run side by side and share its gathered source tensors in L2;
                                     // 2 as 1 with each class's tiles longest list first (the
                                     // short boundary tiles fill the end of the launch);
                                     // -1 automatic: 2 for 64- and 32-bit cores, 0 for bfloat16
};

// Groups of target leaves for the leaf-column near kernel: lpc leaves per
// group (Morton order) and the union of their near offsets.
struct NearGroups {
  int lpc = 0;
  bool ok = false;                   // every member's near list = group list inside the domain
  int64_t ngroups = 0, maxlist = 0;
  DevBuf mem;                        // [ngroups][lpc] leaves (-1 = empty slot)
  DevBuf ptr;                        // [ngroups + 1] into off
  DevBuf off;                        // int4 (dx, dy, dz, 0) per entry
};

struct NearLeavesShape {
  bool ok = false;
  int lpc = 0, tpw = 8, ks = 1, ct = 1;
  size_t parts_bytes = 0;
};

// Transfer data of a handle from htlr_build_quasi (defined with its kernels).
struct QuasiData;

struct htlr_matrix_impl {
  int d = 0, n = 0, p = 0, leaf = 0, L = 0, P = 0, kid = 0;
  int64_t N = 0;
  bool uniform = false;
  double eta2 = 1.0;
  int adm_kind = 0, gl_order = 0, precisions = 7;
  int orth = 0;                      // Alg. 4.1's QR step: 0 none, 1 QR, 2 QRCP (truncated)
  double rank_tol = 1e-13;
  int rank = 0;                      // largest level rank (P = rank^d); each level keeps its own
  double h = 0, w0 = 0, D0 = 0;
  int device = 0;
  Grid grid;
  Plan plan;
  DevBuf x64, x32, w64, w32;         // per-dimension nodes and cell lengths
  DevBuf a64, a32;                   // a(x_i), N values
  DevBuf D64, D32;                   // tensor grids: per-point diagonal integrals
  DevBuf near_ptr, near_src;         // inadmissible leaves (level L)
  DevBuf T64, T32;                   // uniform radial kernels: near-field table by squared distance
  int Tsize = 0;
  std::vector<LevelData> levels;     // index = level
  std::vector<NearGroups> ngroups;   // leaf-column near kernel work lists, per leaves per group
  // near field as class tiles of the matrix-core core apply (uniform 3D grids,
  // 8^3-point leaves): one 512 x 512 block per near offset, built on first use,
  // as a level of its own (index L + 1, so its K-split buffer is its own)
  std::unique_ptr<LevelData> near_lv;
  DevBuf near_w, near_h, near_zero;  // leaf-major u and near result [leaf][rhs][512]; zero tensor
  DevBuf near_off;                   // int4 near offsets, for building each precision's blocks
  size_t device_bytes = 0;
  std::mutex ws_mu;
  Workspace ws;
  Profiler prof;
  std::map<std::pair<int, int>, TuneParams> tune;   // (nrhs, precision) -> choices
  TuneParams cur;                    // choices of the product being issued
  hipEvent_t ev_fork = nullptr;      // level concurrency: fork from and join into the caller's stream
  hipEvent_t ev_level[kMaxLevels] = {};
  std::vector<hipStream_t> side;     // the handle's own side streams for the level chains
  std::shared_ptr<QuasiData> quasi;  // set on quasi-uniform handles: T Ahat S (Sec. 3.3)
  htlr_matrix_impl() = default;
  htlr_matrix_impl(const htlr_matrix_impl&) = delete;
  htlr_matrix_impl& operator=(const htlr_matrix_impl&) = delete;
  ~htlr_matrix_impl() {
    for (hipStream_t s : side) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    for (hipEvent_t e : ev_level)
      if (e) (void)hipEventDestroy(e);
  }
};

// Brackets one launch with events when the handle's profiler is on.
struct ProfScope {
  Profiler& p;
  hipStream_t st;
  bool on;
  Profiler::Rec rec;
  ProfScope(htlr_matrix_impl& A, const char* name, int level, hipStream_t s, bool enable = true)
      : p(A.prof), st(s), on(A.prof.on && enable) {
    if (!on) return;
    rec.name = level >= 0 ? std::string(name) + "_l" + std::to_string(level) : std::string(name);
    rec.a = p.get();
    rec.b = p.get();
    HTLR_HIP(hipEventRecord(rec.a, st));
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(rec.b, st);
    p.recs.push_back(rec);
  }
};

bool core_mfma_ok(const htlr_matrix_impl& A, const LevelData& lv, int prec);
bool core_mfma_any(const htlr_matrix_impl& A, int prec);
// Work-item order of the matrix-core core apply for this precision (the
// choice in A.cur, or the automatic one).
int core_item_order(const htlr_matrix_impl& A, int prec);
// Side streams for the concurrent level chains of a product (a few per
// handle, default priority, non-blocking, created on first use and
// destroyed with the handle, so that the far fields of different handles do
// not queue behind each other); also creates the handle's fork and level
// events.
const std::vector<hipStream_t>& side_streams(htlr_matrix_impl& A);
void ensure_workspace(htlr_matrix_impl& A, int nrhs, int prec);
// Allocates every buffer products with up to nrhs right-hand sides can need
// (work buffers, matrix-core work lists, K-split partial sums), then freezes
// them, so that later products never allocate (graph capture, serving).
void reserve_workspace(htlr_matrix_impl& A, int nrhs);
// Choices for a product of this shape: exact match, else the nearest tuned
// smaller width of the same precision, else the defaults.
TuneParams find_tune(const htlr_matrix_impl& A, int nrhs, int prec);
// Near field on the matrix-core core apply (uniform 3D grids, 8^3-point
// leaves, radial kernels): whether it serves a product of this shape, and the
// product's near field and diagonal term (overwrites f).
bool near_tiles_ok(const htlr_matrix_impl& A, int nrhs);
template <typename T>
void launch_near_tiles(htlr_matrix_impl& A, const T* u, T* f, int nrhs, hipStream_t st);
// Leaf-column near field (uniform 3D grids, 8^3-point leaves, radial kernels, nrhs <= 16).
bool near_leaves_ok(const htlr_matrix_impl& A, int nrhs, int prec);
NearLeavesShape near_leaves_shape(htlr_matrix_impl& A, int nrhs, int prec, bool frozen);
// Whether the product of this shape, with the choices in A.cur, takes the leaf-column near kernel.
bool use_near_leaves(htlr_matrix_impl& A, int nrhs, int prec, bool frozen);
template <typename T>
void launch_near_leaves(htlr_matrix_impl& A, const T* u, T* f, int nrhs, int prec, hipStream_t st);
void launch_core_mfma(htlr_matrix_impl& A, LevelData& lv, int prec, const void* W, void* H, const void* zero,
                      int nrhs, hipStream_t st);
// Near field on uniform 2D grids with a radial kernel and leaves of 8 or 16
// points per side: VALU kernel reusing each (row, row) block's 2m - 1 table values.
bool near_rows2d_ok(const htlr_matrix_impl& A, int nrhs, int prec);
template <typename T>
void launch_near_rows2d(htlr_matrix_impl& A, const T* u, T* f, int nrhs, hipStream_t st);
// Near field on uniform 3D grids with a radial kernel and leaves of 4 points per side.
bool near_rows3d_ok(const htlr_matrix_impl& A, int nrhs, int prec);
template <typename T>
void launch_near_rows3d(htlr_matrix_impl& A, const T* u, T* f, int nrhs, hipStream_t st);
// Work buffers of a product of this shape (handles from htlr_build).
size_t workspace_bytes(const htlr_matrix_impl& A, int nrhs, int prec);
// Column table of a grouped up contraction or down expansion over several
// matrices that share their factors (same d, n, p, leaf on a uniform grid):
// global column r of the launch belongs to the matrix whose work buffer
// (W for the up contraction, H for the down expansion) starts at base[r],
// with ld[r] columns per box, as its column rl[r].  Lives in device memory.
constexpr int kMaxGroupCols = 64;
struct ColTab {
  void* base[kMaxGroupCols];
  int ld[kMaxGroupCols];
  int rl[kMaxGroupCols];
};

// f = A_g u for several matrices with the same factors (uniform grids of
// the same d, n, leaf and Tucker rank; e.g. different kernels): columns
// [c0_g, c0_g + cols[g]) of the column-major N x C buffers u and f belong to
// matrix g, in list order.  The up contraction and down expansion of each
// level whose kernel is a one-pass box kernel, for every matrix's own
// product and for the whole group, run as one launch over all C columns
// (column tables route each column's W and H to its matrix's work buffers);
// the rest runs per matrix.  Everything is issued on st in the single
// product's order (up, core, near field, then down expansions in level
// order), so each column equals its matrix's own product with the same
// kernel choices.  tab_host (pinned) and tab_dev hold 2 * kMaxLevels tables,
// which must stay untouched until st reaches this point.  Takes each
// matrix's work-buffer lock; returns the number of grouped launches.
int product_group(const std::vector<htlr_matrix_impl*>& As, const std::vector<int>& cols, const void* u, void* f,
                  int prec, hipStream_t st, ColTab* tab_host, ColTab* tab_dev);

// Work buffers of one product: per level the source tensors W, the core
// apply's outputs H and the partial up contractions UP, plus the zero source
// tensor of the matrix-core kernel.  noalloc: the buffers live in memory the
// caller provides, and the product takes only kernels that need no lazily
// built work lists, side streams or profiler events (the CSR core apply,
// near-field kernels without K-split partial sums), with the built-in
// choices and every launch on the caller's stream.
struct WorkView {
  void* W[kMaxLevels] = {};
  void* H[kMaxLevels] = {};
  void* UP[kMaxLevels] = {};
  const void* zero = nullptr;
  bool noalloc = false;
};
// f = A u with the work buffers of wv (the caller holds A.ws_mu).
void product_view(htlr_matrix_impl& A, const void* u, void* f, int nrhs, int prec, hipStream_t st,
                  const WorkView& wv);
// Lays the work buffers of a product with nrhs right-hand sides out in one
// region starting at base (256-byte aligned pieces); returns its size in
// bytes.  base NULL: size only.
size_t carve_workview(const htlr_matrix_impl& A, int nrhs, char* base, WorkView* wv);
// f = A u on a handle from htlr_build (work buffers on demand); the caller
// holds A.ws_mu.  u, f: f64 for FP64, f32 otherwise.
void product(htlr_matrix_impl& A, const void* u, void* f, int nrhs, int prec, hipStream_t st);
// Quasi-uniform handles: the uniform-grid matrix Ahat, the product
// f = a o u + T Ahat S u (the caller holds A.ws_mu), and the transfer
// buffers a product of this shape adds to Ahat's work buffers.
htlr_matrix_impl& quasi_inner(htlr_matrix_impl& A);
void quasi_matvec(htlr_matrix_impl& A, const void* u, void* f, int nrhs, int prec, hipStream_t st);
size_t quasi_buffer_bytes(const htlr_matrix_impl& A, int nrhs, int prec);

}  // namespace htlr

struct htlr_matrix_s : htlr::htlr_matrix_impl {};
