// Near field + diagonal on the matrix cores with target leaves as GEMM
// columns (uniform 3D grid, leaves of 8^3 points, radial kernel).
//
// The near part of the product (Alg. 4.2, the inadmissible leaves of the
// block cluster tree) is f_tau += sum_{sigma in near(tau)} K_{tau,sigma}
// u_sigma.  On a uniform grid the block K_{tau,sigma} depends only on the
// leaf offset Delta = sigma - tau: its entry (i, j) is the kernel at the
// point displacement 8 (tau - sigma) + (i - j), a value of the table T of
// kernel values by integer squared distance (T[0] holds the singular cell
// integral).  So the blocks of all target leaves with the same Delta are one
// matrix, and a group of target leaves can share every kernel value:
//
//   rows     i            (512 target points of a leaf),
//   columns  (tau, r)     (the leaves of a group x right-hand sides),
//   K        (Delta, j)   (offsets of the group x 512 source points),
//
// with B[(Delta, j), (tau, r)] = u_r at point j of leaf tau + Delta, or zero
// when that leaf lies outside the domain.  One 16x16x4 MFMA then does 1024
// multiply-adds for one table read and one staged source value per lane,
// where a row-per-lane VALU loop needs a table read for every few
// multiply-adds; with two 16-column tiles per wave each gathered value feeds
// two MFMAs.  A group holds 16 CT / nrhs leaves with equal or similar near
// offset lists (sorted by list, then Morton order), and its offset list is
// the union of its members' (checked on the host to equal each member's own
// list inside the domain).
//
// Work item = (group, row block, K split); split s > 0 writes its partial
// sum to a separate buffer and a reduction adds the parts in split order and
// the diagonal a(x_i) u_i, so the result is deterministic.

#include <algorithm>
#include <array>
#include <set>

#include "htlr_device.h"
#include "htlr_handle.h"

namespace htlr {

namespace {

typedef float nl_f32x4 __attribute__((ext_vector_type(4)));
typedef double nl_f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t nl_lin3(int i0, int i1, int i2, int n) {
  return (int64_t)i0 + (int64_t)n * ((int64_t)i1 + (int64_t)n * i2);
}

// Column descriptor: target leaf coordinates and rhs, or x = -1 (empty).
struct NlCol { int x, y, z, r; };

// Staging: 2048 (source point, column) values per round, i.e. 128 source
// points for 16 columns or 64 for 32; rows padded by one element.  The next
// round is loaded into registers while the current one is computed.
template <int CT> struct NlStage {
  static constexpr int NC = 16 * CT;          // columns
  static constexpr int JH = 2048 / NC;        // source points per round
  static constexpr int LDU = NC + 1;          // padded row of the staged sources
};

// TPW 16-row MFMA tiles per wave, CT 16-column tiles (each gathered kernel
// value feeds CT MFMAs); 4 waves; a workgroup covers 64 * TPW rows.
template <typename T, int TPW, int CT>
__global__ __launch_bounds__(256) void k_near_leaves(
    const T* __restrict__ u, T* __restrict__ out, const T* __restrict__ a, const int32_t* __restrict__ gmem,
    const int64_t* __restrict__ gptr, const int4* __restrict__ goff, const T* __restrict__ table, int tsize, int n,
    int B, int nrhs, int lpc, int64_t ngroups, int ksplit, int64_t part_stride) {
  using V4 = typename std::conditional<std::is_same<T, double>::value, nl_f64x4, nl_f32x4>::type;
  using S = NlStage<CT>;
  constexpr int NC = S::NC, JH = S::JH, LDU = S::LDU;
  constexpr int RB = 64 * TPW;           // rows per workgroup
  constexpr int NRB = 512 / RB;          // row blocks per leaf
  constexpr int TZ = TPW / 4;            // distinct z rows of a lane's tiles
  constexpr int CPT = NC * JH / 256;     // staged values per thread per round (8)
  static_assert(TPW == 4 || TPW == 8, "4 or 8 tiles per wave");
  static_assert(CT == 1 || CT == 2, "one or two column tiles");
  extern __shared__ unsigned char smem_raw[];
  T* tab = reinterpret_cast<T*>(smem_raw);
  const int tpad = (tsize + 3) & ~3;
  T* us = tab + tpad;                                       // [JH][LDU]
  NlCol* ccol = reinterpret_cast<NlCol*>(us + JH * LDU);    // [NC]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

  // Work items are dealt to the 8 XCDs round robin; consecutive items (one
  // group) land on one XCD, so their source leaves are shared in its L2.
  const int64_t nitems = ngroups * NRB * ksplit;
  const int64_t per_xcd = (nitems + 7) / 8;
  const int64_t q = (int64_t)(blockIdx.x % 8) * per_xcd + (int64_t)(blockIdx.x / 8);
  if (q >= nitems) return;
  const int split = (int)(q % ksplit);
  const int rb = (int)((q / ksplit) % NRB);
  const int64_t grp = q / ((int64_t)ksplit * NRB);

  for (int s = tid; s < tsize; s += 256) tab[s] = table[s];
  if (tid < NC) {
    const int lc = tid / nrhs, r = tid % nrhs;
    NlCol c{-1, 0, 0, 0};
    if (lc < lpc) {
      const int t = gmem[grp * lpc + lc];
      if (t >= 0) c = NlCol{t % B, (t / B) % B, t / (B * B), r};
    }
    ccol[tid] = c;
  }
  __syncthreads();

  int64_t e0 = gptr[grp], e1 = gptr[grp + 1];
  {
    const int64_t chunk = (e1 - e0 + ksplit - 1) / ksplit;
    const int64_t lo = e0 + split * chunk;
    e1 = lo + chunk < e1 ? lo + chunk : e1;
    e0 = lo < e1 ? lo : e1;
  }

  // rows of this lane: i = wbase + 16 t + l15, t < TPW
  const int l15 = lane & 15, jl = lane >> 4;
  const int wbase = rb * RB + wv * 16 * TPW;
  const int ix = l15 & 7;
  int iy[4], iz[TZ];
#pragma unroll
  for (int k = 0; k < 4; ++k) iy[k] = (2 * k + (l15 >> 3)) & 7;
#pragma unroll
  for (int k = 0; k < TZ; ++k) iz[k] = (wbase >> 6) + k;

  V4 acc[TPW][CT];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[t][c] = V4{T(0), T(0), T(0), T(0)};

  const int64_t N = (int64_t)n * n * n;
  // staged value k of this thread: source point jj of the round, column cs + k * (256 / JH)
  const int jj = tid % JH, cs = tid / JH;
  constexpr int NR = 512 / JH;            // rounds per offset
  T pre[CPT];                              // the next round, loaded ahead
#define NL_LOAD(OFF, RND)                                                                              \
  {                                                                                                    \
    const int j_ = (RND) * JH + jj;                                                                    \
    const int jx_ = j_ & 7, jy_ = (j_ >> 3) & 7, jz_ = j_ >> 6;                                        \
    _Pragma("unroll") for (int k = 0; k < CPT; ++k) {                                                  \
      const NlCol cc = ccol[cs + k * (256 / JH)];                                                      \
      const int sx = cc.x + (OFF).x, sy = cc.y + (OFF).y, sz = cc.z + (OFF).z;                         \
      const bool ok = cc.x >= 0 && sx >= 0 && sx < B && sy >= 0 && sy < B && sz >= 0 && sz < B;        \
      pre[k] = ok ? u[(int64_t)cc.r * N + nl_lin3(sx * 8 + jx_, sy * 8 + jy_, sz * 8 + jz_, n)] : T(0); \
    }                                                                                                  \
  }
  if (e0 < e1) {
    const int4 o0 = goff[e0];
    NL_LOAD(o0, 0);
  }
  for (int64_t e = e0; e < e1; ++e) {
    const int4 o = goff[e];
    // point displacement I - J = (i - j) - 8 Delta, per dimension
    const int cx = ix - 8 * o.x;
    int cy[4], cz[TZ];
#pragma unroll
    for (int k = 0; k < 4; ++k) cy[k] = iy[k] - 8 * o.y;
#pragma unroll
    for (int k = 0; k < TZ; ++k) cz[k] = iz[k] - 8 * o.z;
    for (int round = 0; round < NR; ++round) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < CPT; ++k) us[jj * LDU + cs + k * (256 / JH)] = pre[k];
      __syncthreads();
      if (round + 1 < NR) {
        NL_LOAD(o, round + 1);
      } else if (e + 1 < e1) {
        const int4 on = goff[e + 1];
        NL_LOAD(on, 0);
      }
      const T* ub = us + l15;
      // the round's source points are whole x-lines: JH / 8 lines, 2 K steps each
      for (int line = 0; line < JH / 8; ++line) {
        const int jabs = round * JH + line * 8;      // first point of the line
        const int jy = (jabs >> 3) & 7, jz = jabs >> 6;
        int dyz[TPW];
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
          const int dy = cy[t & 3] - jy, dz = cz[t >> 2] - jz;
          dyz[t] = dy * dy + dz * dz;
        }
#pragma unroll
        for (int xh = 0; xh < 2; ++xh) {
          const int jx = 4 * xh + jl;
          const int dx = cx - jx;
          const int dx2 = dx * dx;
          const int jloc = line * 8 + jx;              // staged row of this lane's source
          T b[CT];
#pragma unroll
          for (int c = 0; c < CT; ++c) b[c] = ub[jloc * LDU + 16 * c];
#pragma unroll
          for (int t = 0; t < TPW; ++t) {
            const T av = tab[dx2 + dyz[t]];
#pragma unroll
            for (int c = 0; c < CT; ++c) {
              if constexpr (std::is_same<T, double>::value)
                acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b[c], acc[t][c], 0, 0, 0);
              else
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b[c], acc[t][c], 0, 0, 0);
            }
          }
        }
      }
    }
  }
#undef NL_LOAD

  // write the owned tiles: f (single split, with the diagonal) or a partial sum
  T* o = out + (ksplit > 1 ? (int64_t)split * part_stride : 0);
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const NlCol cc = ccol[16 * c + l15];
    if (cc.x < 0) continue;
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // accumulator layouts of 16x16x4: f32 register v holds row 4 (lane/16) + v,
        // f64 register v holds row lane/16 + 4 v; the column is lane % 16
        const int row = std::is_same<T, double>::value ? jl + 4 * v : 4 * jl + v;
        const int i = wbase + 16 * t + row;
        const int64_t g = nl_lin3(cc.x * 8 + (i & 7), cc.y * 8 + ((i >> 3) & 7), cc.z * 8 + (i >> 6), n);
        const int64_t idx = (int64_t)cc.r * N + g;
        o[idx] = ksplit > 1 ? acc[t][c][v] : acc[t][c][v] + a[g] * u[idx];
      }
  }
}

// f = sum of the K-split parts in split order + a(x_i) u_i.
template <typename T>
__global__ void k_near_leaves_reduce(const T* __restrict__ parts, int ksplit, int64_t stride, T* __restrict__ f,
                                     const T* __restrict__ a, const T* __restrict__ u, int64_t N, int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    T v = parts[i];
    for (int s = 1; s < ksplit; ++s) v += parts[s * stride + i];
    f[i] = v + a[i % N] * u[i];
  }
}

uint64_t nl_morton3(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t m = 0;
  for (int b = 0; b < 21; ++b)
    m |= ((uint64_t)((x >> b) & 1) << (3 * b)) | ((uint64_t)((y >> b) & 1) << (3 * b + 1)) |
         ((uint64_t)((z >> b) & 1) << (3 * b + 2));
  return m;
}

size_t nl_lds_bytes(const htlr_matrix_impl& A, size_t esz, int ct) {
  const size_t stage = ct == 2 ? (size_t)NlStage<2>::JH * NlStage<2>::LDU : (size_t)NlStage<1>::JH * NlStage<1>::LDU;
  return (((size_t)A.Tsize + 3) & ~size_t(3)) * esz + stage * esz + 16 * ct * sizeof(NlCol);
}

// Groups of lpc leaves, built on first use; nullptr when some leaf's near
// list is not the group's offset list restricted to the domain.
NearGroups* groups_for(htlr_matrix_impl& A, int lpc, bool frozen) {
  for (auto& g : A.ngroups)
    if (g.lpc == lpc) return g.ok ? &g : nullptr;
  if (frozen) fail(HTLR_ERR_INVALID, "near-field work lists were not reserved");
  NearGroups G;
  G.lpc = lpc;
  const int B = A.plan.B[A.L];
  const Csr& nc = A.plan.near;
  // Leaves ordered by their list of near offsets, then in Morton order: a
  // group's offset list is the union of its members' lists, so leaves near
  // the same faces, edges or corners of the domain are grouped together.
  const int64_t nleaf = (int64_t)B * B * B;
  std::vector<std::vector<std::array<int, 3>>> lists(nleaf);
  for (int64_t t = 0; t < nleaf; ++t) {
    const int tx = (int)(t % B), ty = (int)((t / B) % B), tz = (int)(t / ((int64_t)B * B));
    for (int64_t e = nc.ptr[t]; e < nc.ptr[t + 1]; ++e) {
      const int32_t sg = nc.src[e];
      lists[t].push_back({sg % B - tx, (sg / B) % B - ty, sg / (B * B) - tz});
    }
    std::sort(lists[t].begin(), lists[t].end());
  }
  std::vector<std::pair<uint64_t, int32_t>> leaves;
  for (int64_t t = 0; t < nleaf; ++t)
    leaves.push_back({nl_morton3((uint32_t)(t % B), (uint32_t)((t / B) % B), (uint32_t)(t / ((int64_t)B * B))),
                      (int32_t)t});
  std::sort(leaves.begin(), leaves.end(), [&](const std::pair<uint64_t, int32_t>& x,
                                              const std::pair<uint64_t, int32_t>& y) {
    if (lists[x.second] != lists[y.second]) return lists[x.second] < lists[y.second];
    return x.first < y.first;
  });
  std::vector<int32_t> mem;
  std::vector<int64_t> ptr{0};
  std::vector<int4> off;
  bool ok = true;
  for (size_t s = 0; s < leaves.size() && ok; s += lpc) {
    std::set<std::array<int, 3>> offs;
    std::vector<int32_t> members;
    for (size_t q = s; q < std::min(leaves.size(), s + (size_t)lpc); ++q) {
      const int32_t t = leaves[q].second;
      members.push_back(t);
      const int tx = t % B, ty = (t / B) % B, tz = t / (B * B);
      for (int64_t e = nc.ptr[t]; e < nc.ptr[t + 1]; ++e) {
        const int32_t sg = nc.src[e];
        offs.insert({sg % B - tx, (sg / B) % B - ty, sg / (B * B) - tz});
      }
    }
    for (int32_t t : members) {
      const int tx = t % B, ty = (t / B) % B, tz = t / (B * B);
      int64_t inside = 0;
      for (auto& o : offs) {
        const int sx = tx + o[0], sy = ty + o[1], sz = tz + o[2];
        if (sx >= 0 && sx < B && sy >= 0 && sy < B && sz >= 0 && sz < B) ++inside;
      }
      if (inside != nc.ptr[t + 1] - nc.ptr[t]) ok = false;
    }
    for (int q = 0; q < lpc; ++q) mem.push_back(q < (int)members.size() ? members[q] : -1);
    for (auto& o : offs) off.push_back(make_int4(o[0], o[1], o[2], 0));
    ptr.push_back((int64_t)off.size());
    G.maxlist = std::max<int64_t>(G.maxlist, (int64_t)offs.size());
  }
  G.ok = ok;
  if (ok) {
    G.ngroups = (int64_t)ptr.size() - 1;
    G.mem.alloc(mem.size() * sizeof(int32_t));
    G.ptr.alloc(ptr.size() * sizeof(int64_t));
    G.off.alloc(std::max<size_t>(off.size(), 1) * sizeof(int4));
    HTLR_HIP(hipMemcpy(G.mem.ptr, mem.data(), mem.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HTLR_HIP(hipMemcpy(G.ptr.ptr, ptr.data(), ptr.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    if (!off.empty()) HTLR_HIP(hipMemcpy(G.off.ptr, off.data(), off.size() * sizeof(int4), hipMemcpyHostToDevice));
  }
  A.ngroups.push_back(std::move(G));
  return ok ? &A.ngroups.back() : nullptr;
}

}  // namespace

bool near_leaves_ok(const htlr_matrix_impl& A, int nrhs, int prec) {
  const size_t esz = prec == HTLR_FP64 ? 8 : 4;
  return A.uniform && A.d == 3 && A.plan.m[A.L] == 8 && A.kid != HTLR_K_POLY_TEST && nrhs >= 1 && nrhs <= 16 &&
         nl_lds_bytes(A, esz, 1) <= 64 * 1024 && nl_lds_bytes(A, esz, 2) <= 64 * 1024;
}

// Tiles per wave and K splits of the leaf-column near kernel.
NearLeavesShape near_leaves_shape(htlr_matrix_impl& A, int nrhs, int prec, bool frozen) {
  NearLeavesShape s;
  (void)prec;
  s.ct = A.cur.near_ct == 2 ? 2 : 1;
  s.lpc = 16 * s.ct / nrhs;
  if (s.lpc < 1) return s;
  NearGroups* G = groups_for(A, s.lpc, frozen);
  if (!G) return s;
  s.ok = true;
  s.tpw = A.cur.near_tpw == 4 ? 4 : 8;
  const int64_t base = G->ngroups * (512 / (64 * s.tpw));
  if (A.cur.near_ks > 0) {
    s.ks = A.cur.near_ks;
  } else {
    // aim for about 768 workgroups (3 per CU, as the LDS allows), at least 4 offsets per split
    s.ks = (int)std::max<int64_t>(1, std::min<int64_t>((768 + base / 2) / std::max<int64_t>(base, 1),
                                                       std::max<int64_t>(G->maxlist / 4, 1)));
  }
  s.ks = (int)std::max<int64_t>(1, std::min<int64_t>(s.ks, std::max<int64_t>(G->maxlist, 1)));
  s.parts_bytes = s.ks > 1 ? (size_t)s.ks * A.N * nrhs * (prec == HTLR_FP64 ? 8 : 4) : 0;
  return s;
}

bool use_near_leaves(htlr_matrix_impl& A, int nrhs, int prec, bool frozen) {
  if (!near_leaves_ok(A, nrhs, prec)) return false;
  // automatic choice up to 8 right-hand sides; above, only when tuned
  if (!(A.cur.near_kind == 2 || (A.cur.near_kind < 0 && nrhs <= 8))) return false;
  return near_leaves_shape(A, nrhs, prec, frozen).ok;
}

template <typename T>
void launch_near_leaves(htlr_matrix_impl& A, const T* u, T* f, int nrhs, int prec, hipStream_t st) {
  const NearLeavesShape s = near_leaves_shape(A, nrhs, prec, A.ws.frozen);
  if (!s.ok) fail(HTLR_ERR_UNSUPPORTED, "near lists are not translation invariant");
  NearGroups* G = groups_for(A, s.lpc, A.ws.frozen);
  const bool f64 = std::is_same<T, double>::value;
  const T* tab = f64 ? (const T*)A.T64.ptr : (const T*)A.T32.ptr;
  const T* a = f64 ? (const T*)A.a64.ptr : (const T*)A.a32.ptr;
  const int B = A.plan.B[A.L];
  const int64_t total = A.N * nrhs;
  T* out = f;
  if (s.ks > 1) {
    if (A.ws.nparts.bytes < s.parts_bytes) {
      if (A.ws.frozen) fail(HTLR_ERR_INVALID, "near-field partial buffer exceeds the reserved size");
      A.ws.nparts.alloc(s.parts_bytes);
    }
    out = A.ws.nparts.as<T>();
  }
  const int64_t nitems = G->ngroups * (512 / (64 * s.tpw)) * s.ks;
  const int64_t grid = (nitems + 7) / 8 * 8;
  if (grid > 0x7fffffff) fail(HTLR_ERR_UNSUPPORTED, "near-field work list too large");
  const size_t sh = nl_lds_bytes(A, sizeof(T), s.ct);
#define HTLR_NL(TPWV, CTV)                                                                                      \
  hipLaunchKernelGGL((k_near_leaves<T, TPWV, CTV>), dim3((unsigned)grid), dim3(256), sh, st, u, out, a,        \
                     G->mem.as<int32_t>(), G->ptr.as<int64_t>(), G->off.as<int4>(), tab, A.Tsize, A.n, B, nrhs, \
                     s.lpc, G->ngroups, s.ks, total)
  if (s.tpw == 4) {
    if (s.ct == 2) HTLR_NL(4, 2); else HTLR_NL(4, 1);
  } else {
    if (s.ct == 2) HTLR_NL(8, 2); else HTLR_NL(8, 1);
  }
#undef HTLR_NL
  HTLR_HIP(hipGetLastError());
  if (s.ks > 1) {
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_near_leaves_reduce<T>, dim3(blocks), dim3(256), 0, st, (const T*)out, s.ks, total, f, a, u,
                       A.N, total);
    HTLR_HIP(hipGetLastError());
  }
}

template void launch_near_leaves<double>(htlr_matrix_impl&, const double*, double*, int, int, hipStream_t);
template void launch_near_leaves<float>(htlr_matrix_impl&, const float*, float*, int, int, hipStream_t);

}  // namespace htlr
