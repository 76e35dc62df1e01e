// Core apply on the matrix cores (uniform grids).
//
// For one level, H_tau = sum_{sigma in adm(tau)} G_{sigma - tau} W_sigma
// (Alg. 4.2: H = G x_{[d+1..2d],[1..d]} W, summed over the admissible leaves
// of a row block).  On a uniform grid the cores depend only on the offset
// Delta = sigma - tau, and the admissible offsets of a box depend only on its
// parity class (tau mod 2, which fixes the parent offsets of Def. 2.4) and on
// the domain boundary.  So a set of boxes of one class shares one list of
// offsets, and the level becomes an implicit GEMM:
//
//   rows    t          (p^d core rows),
//   columns (tau, r)   (boxes of a tile x right-hand sides),
//   K       (Delta, s) (offsets of the tile x p^d core columns),
//
// with the B operand gathered from W_{tau + Delta}; a column whose source box
// falls outside the domain reads a zero tensor.  Each workgroup owns a
// 128 x 128 output tile and accumulates it over the tile's whole K range
// (owner computes, no atomics, deterministic).  Operands are staged through
// LDS in 64- or 128-byte K slices with double buffering; 4 waves each compute a
// 64 x 64 sub-tile with 32x32 (bf16, f32) or 16x16 (f64) MFMA instructions.

#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <set>

#include "htlr_device.h"
#include "htlr_handle.h"

namespace htlr {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));   // one 16-byte staged chunk

constexpr int kBNmax = 128;  // right-hand sides a matrix-core column tile can hold

template <typename TE> struct AccT { using type = float; };
template <> struct AccT<double> { using type = double; };

// Operand pointers are kept in the global address space from the kernel
// entry on: pointers selected and carried across loop iterations otherwise
// become generic, and generic loads are also counted by the LDS wait counter,
// which would make every LDS wait of the MFMA loop wait for the prefetch.
template <typename T> using gptr = const __attribute__((address_space(1))) T*;
typedef __attribute__((address_space(3))) void* lds_vptr;

// One direct-to-LDS load: each lane's 16 bytes at src go to LDS byte address
// lds + 16 * lane (lds wave-uniform).  Written as a statement of its own so
// that the compiler, which cannot tell which LDS buffer such a load writes,
// does not make the operand reads of the other buffer wait for it; the
// caller waits for the load counter before the barrier that publishes the
// buffer.  The instruction has no register result (its address registers
// are read at issue).
// M0 (the LDS base of the load) is written here and declared clobbered; no
// other code of these kernels keeps a value in M0.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void lds_dma16(const void* src, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "s"(lds)
               : "memory", "m0");
}
#pragma clang diagnostic pop

// Source tensor of one staged column for offset o, or the zero tensor when
// the column is empty or its source box lies outside the domain.
template <typename TE>
__device__ __forceinline__ gptr<TE> col_src(gptr<TE> W, gptr<TE> zero, int ct, int cx, int cy, int cz, int cr,
                                            int4 o, int B, int nrhs, int P) {
  const int sx = cx + o.y, sy = cy + o.z, sz = cz + o.w;
  const bool ok = ct >= 0 && sx >= 0 && sx < B && sy >= 0 && sy < B && sz >= 0 && sz < B;
  const int64_t sg = (int64_t)sx + (int64_t)B * (sy + (int64_t)B * sz);
  return ok ? W + (sg * nrhs + cr) * P : zero;
}

// Bytes of K staged per row and stage: 128 for the 32-bit and 64-bit tiles
// (more bytes in flight per stage while the next one is fetched), 64 for
// bfloat16 and the 256-row tile (LDS and registers).
template <typename TE, int BMT, int BNT>
constexpr int stage_bytes() {
  return (sizeof(TE) >= 4 && BMT == 128 && !(sizeof(TE) == 8 && BNT == 64)) ? 128 : 64;
}

// Rows per wave: 64, or 112 (seven 16-row f64 MFMA tiles) for the 224-row
// tile, which holds p^d = 216 (p = 6, d = 3) core rows in one block.
constexpr int core_wave_rows(int bmt) { return bmt == 224 ? 112 : 64; }
constexpr int core_threads(int bmt) { return 128 * (bmt / core_wave_rows(bmt)); }

// Stages in flight per thread (1 or 2): 2 where the extra register slot
// keeps the same number of waves per SIMD.
template <typename TE, int BMT, int BNT>
constexpr int prefetch_depth() {
  return (sizeof(TE) == 8) ? 1 : 2;
}

// BMT x BNT output tile per workgroup; waves arranged (BMT / WR) x 2, each
// owning WR rows x BNT/2 columns (WR = core_wave_rows(BMT)).
template <typename TE, int BMT, int BNT>
__global__ __launch_bounds__(core_threads(BMT)) __attribute__((amdgpu_waves_per_eu(2))) void k_core_mfma(
    const TE* __restrict__ G, const TE* __restrict__ W, const TE* __restrict__ zero,
    typename AccT<TE>::type* __restrict__ H, const int32_t* __restrict__ tile_tau,
    const int64_t* __restrict__ tile_ptr, const int4* __restrict__ tile_off, const int32_t* __restrict__ items,
    int nitems, int ksplit, int64_t part_stride, int P, int nrhs, int NB, int B, const int32_t* __restrict__ tile_out) {
  using TA = typename AccT<TE>::type;
  const gptr<TE> Gg = (gptr<TE>)G, Wg = (gptr<TE>)W, zg = (gptr<TE>)zero;
  constexpr int NT = core_threads(BMT);   // threads
  constexpr int WR = core_wave_rows(BMT); // rows per wave
  constexpr int E = 16 / sizeof(TE);      // elements per 16-byte chunk
  constexpr int CB = stage_bytes<TE, BMT, BNT>();
  constexpr int PD = prefetch_depth<TE, BMT, BNT>();
  constexpr int KBE = CB / sizeof(TE);    // K elements per stage
  // FP64 128 x 128 tiles stage by direct-to-LDS loads (global loads with an
  // LDS destination: no register staging, no LDS writes by the waves).  One
  // such load writes 64 consecutive 16-byte chunks, so the rows are unpadded
  // (128 bytes) and a row's chunks are XOR-swizzled by (row / 2) mod 8, which
  // keeps the 16-row operand reads free of bank conflicts.
  constexpr bool DL = std::is_same<TE, double>::value && BMT == 128 && BNT == 128;
  constexpr int LDW = DL ? KBE : KBE + E; // LDS row (padded unless DL)
  constexpr int CPR = CB / 16;            // 16-byte chunks per staged row
  constexpr int RPP = NT / CPR;           // rows staged per pass of all threads
  constexpr int NA = (BMT + RPP - 1) / RPP;   // A rows staged per thread (the last pass may be partial)
  constexpr int NBH = BNT / RPP;          // B columns staged per thread
  constexpr int WNC = BNT / 2;            // columns per wave
  static_assert(NA >= 1 && NBH >= 1 && NBH * RPP == BNT, "staging shape");
  static_assert(!DL || (CPR == 8 && NA * RPP == BMT), "direct-to-LDS staging shape");
  constexpr bool APART = NA * RPP != BMT;     // rows srow + (NA - 1) RPP >= BMT are not staged
  __shared__ __align__(16) TE As[2][BMT * LDW];
  __shared__ __align__(16) TE Bs[2][BNT * LDW];
#define HTLR_AS(BUF) (As[BUF])
#define HTLR_BS(BUF) (Bs[BUF])
  // LDS byte address of a staging position (wave-uniform)
  auto lds_addr = [](const TE* p) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(uintptr_t)(lds_vptr)(TE*)p);
  };

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // Work item of this workgroup.  Workgroups are dealt to the 8 XCDs round
  // robin; consecutive items (one parity class, one row block) go to one XCD
  // so that the workgroups sharing an L2 stream the same cores.
  const int per_xcd = (nitems + 7) / 8;
  const int q = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
  if (q >= nitems) return;
  const int item = items[q];
  const int tile = item >> 12;
  const int m0 = ((item >> 6) & 63) * BMT;
  const int split = item & 63;
  const int part = tid % CPR;             // 16-byte chunk within a staged row slice
  const int srow = tid / CPR;             // staged row / column, plus multiples of RPP
  // K chunk this thread loads: with DL the chunk stored at position `part`
  // of a row (rows srow + i RPP share (row / 2) mod 8 since RPP = 32)
  const int cpart = DL ? (part ^ ((srow >> 1) & 7)) : part;
  const int wbase = __builtin_amdgcn_readfirstlane(wv) * 64;   // first chunk of this wave's lanes

  // columns staged by this thread: target box (or -1), rhs, box coordinates
  int ct[NBH], cr[NBH], cx[NBH], cy[NBH], cz[NBH];
#pragma unroll
  for (int h = 0; h < NBH; ++h) {
    const int col = srow + h * RPP;
    const int b = col / nrhs;
    cr[h] = col % nrhs;
    ct[h] = (b < NB) ? tile_tau[(int64_t)tile * NB + b] : -1;
    const int t = ct[h] < 0 ? 0 : ct[h];
    cx[h] = t % B;
    cy[h] = (t / B) % B;
    cz[h] = t / (B * B);
  }

  int64_t e0 = tile_ptr[tile], e1 = tile_ptr[tile + 1];
  {
    const int64_t chunk = (e1 - e0 + ksplit - 1) / ksplit;
    const int64_t lo = e0 + split * chunk;
    e1 = lo + chunk < e1 ? lo + chunk : e1;
    e0 = lo < e1 ? lo : e1;
  }
  H += split * part_stride;   // partial sums of split > 0 go to separate buffers
  const int ksteps = (P + KBE - 1) / KBE;
  const int64_t nstage = (e1 - e0) * ksteps;
  const int64_t PP = (int64_t)P * P;
  const u32x4 z4 = u32x4{0u, 0u, 0u, 0u};

  gptr<TE> gA = Gg;
  gptr<TE> gB[NBH];
  // two register slots of staged chunks: with prefetch depth 2 the loads of
  // stage s + 2 are in flight while stage s is computed and stage s + 1 is
  // written to LDS
  u32x4 ra0[NA], rb0[NBH], ra1[NA], rb1[NBH];
#pragma unroll
  for (int h = 0; h < NBH; ++h) { gB[h] = zg; rb0[h] = z4; rb1[h] = z4; }
#pragma unroll
  for (int i = 0; i < NA; ++i) { ra0[i] = z4; ra1[i] = z4; }

  const int wm = wv >> 1, wn = wv & 1;
  constexpr bool k16 = std::is_same<TE, double>::value;   // 16x16 tiles for f64
  constexpr int TM = k16 ? 16 : 32;                        // MFMA tile side
  constexpr int TI = WR / TM, TJ = WNC / TM;               // MFMA tiles per wave
  static_assert(TI * TM == WR, "wave rows in whole MFMA tiles");
  using AccV = typename std::conditional<k16, f64x4, f32x16>::type;
  AccV acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = AccV{};

#define HTLR_SET_DELTA(EIDX)                                                                  \
  {                                                                                           \
    const int4 o_ = tile_off[EIDX];                                                           \
    gA = Gg + (int64_t)o_.x * PP;                                                             \
    _Pragma("unroll") for (int h = 0; h < NBH; ++h)                                           \
      gB[h] = col_src<TE>(Wg, zg, ct[h], cx[h], cy[h], cz[h], cr[h], o_, B, nrhs, P);        \
  }
// Out-of-range chunks read the zero tensor (a select between two pointers,
// not between a loaded value and a zero held in memory).
#define HTLR_GLOAD(RA, RB, K0)                                                                           \
  {                                                                                                      \
    const int k_ = (K0) + part * E;                                                                      \
    const bool kin_ = k_ < P;                                                                            \
    _Pragma("unroll") for (int i = 0; i < NA; ++i) {                                                     \
      const int ar_ = m0 + srow + i * RPP;                                                               \
      const bool ain_ = !APART || srow + i * RPP < BMT;                                                  \
      const gptr<TE> pa_ = (kin_ && ain_ && ar_ < P) ? gA + (int64_t)ar_ * P + k_ : zg;                  \
      RA[i] = *(gptr<u32x4>)pa_;                                                                         \
    }                                                                                                    \
    _Pragma("unroll") for (int h = 0; h < NBH; ++h) {                                                    \
      const gptr<TE> pb_ = kin_ ? gB[h] + k_ : zg;                                                       \
      RB[h] = *(gptr<u32x4>)pb_;                                                                         \
    }                                                                                                    \
  }
#define HTLR_SSTORE(RA, RB, BUF)                                                                      \
  {                                                                                                   \
    _Pragma("unroll") for (int i = 0; i < NA; ++i)                                                    \
      if (!APART || srow + i * RPP < BMT)                                                             \
        *reinterpret_cast<u32x4*>(&HTLR_AS(BUF)[(srow + i * RPP) * LDW + part * E]) = RA[i];               \
    _Pragma("unroll") for (int h = 0; h < NBH; ++h)                                                   \
      *reinterpret_cast<u32x4*>(&HTLR_BS(BUF)[(srow + h * RPP) * LDW + part * E]) = RB[h];                 \
  }

// Direct-to-LDS load of the stage at K0 into LDS buffer BUF: lane l of wave
// w writes chunk i NT + 64 w + l, i.e. row srow + i RPP, position part.
#define HTLR_DLOAD(BUF, K0)                                                                              \
  {                                                                                                      \
    const int k_ = (K0) + cpart * E;                                                                     \
    const bool kin_ = k_ < P;                                                                            \
    _Pragma("unroll") for (int i = 0; i < NA; ++i) {                                                     \
      const int ar_ = m0 + srow + i * RPP;                                                               \
      const gptr<TE> pa_ = (kin_ && ar_ < P) ? gA + (int64_t)ar_ * P + k_ : zg;                          \
      lds_dma16((const void*)pa_, lds_addr(&HTLR_AS(BUF)[(i * NT + wbase) * E]));                        \
    }                                                                                                    \
    _Pragma("unroll") for (int h = 0; h < NBH; ++h) {                                                    \
      const gptr<TE> pb_ = kin_ ? gB[h] + k_ : zg;                                                       \
      lds_dma16((const void*)pb_, lds_addr(&HTLR_BS(BUF)[(h * NT + wbase) * E]));                        \
    }                                                                                                    \
  }
#define HTLR_DLOAD_NEXT(BUF)                     \
  {                                              \
    if (++ksL == ksteps) { ksL = 0; ++eL; }      \
    if (ksL == 0) HTLR_SET_DELTA(eL);            \
    HTLR_DLOAD(BUF, ksL * KBE);                  \
  }
// Advance (EL, KSL) to the next stage and load it into (RA, RB).
#define HTLR_LOAD_NEXT(RA, RB)                   \
  {                                              \
    if (++ksL == ksteps) { ksL = 0; ++eL; }      \
    if (ksL == 0) HTLR_SET_DELTA(eL);            \
    HTLR_GLOAD(RA, RB, ksL * KBE);               \
  }
// Schedule of one stage of KS K steps (NR operand reads from LDS and NM
// MFMAs each): the reads of each step are interleaved with the MFMAs of the
// step before, instead of all waiting behind them.  Instruction order only;
// the arithmetic is unchanged.
#define HTLR_PIPELINE(KS, NR, NM)                                                             \
  {                                                                                           \
    if constexpr ((KS) > 1) {                                                                 \
      __builtin_amdgcn_sched_group_barrier(0x100, (NR), 0);                                   \
      _Pragma("unroll") for (int r_ = 0; r_ < (KS) - 1; ++r_) {                               \
        _Pragma("unroll") for (int q_ = 0; q_ < (NR); ++q_) {                                 \
          __builtin_amdgcn_sched_group_barrier(0x008, (NM) / (NR) > 0 ? (NM) / (NR) : 1, 0);  \
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);                                  \
        }                                                                                     \
      }                                                                                       \
      __builtin_amdgcn_sched_group_barrier(0x008, (NM), 0);                                   \
    }                                                                                         \
  }
// Column of this lane's f64 operand element at K step KK within its LDS row
// (16 rows x 4 K columns per read; rows r and the swizzle (r / 2) mod 8 =
// (lane / 2) mod 8, as every wave's rows start at a multiple of 16).
  const int kswz = DL ? ((lane >> 1) & 7) : 0;
  auto kcol = [&](int kk) {
    const int kc = kk + (lane >> 4);
    return DL ? ((((kc >> 1) ^ kswz) << 1) | (kc & 1)) : kc;
  };
#define HTLR_COMPUTE(CUR)                                                                                                        \
  {                                                                                                                        \
      const TE* Asb = HTLR_AS(CUR) + (wm * WR) * LDW;                                                                           \
      const TE* Bsb = HTLR_BS(CUR) + (wn * WNC) * LDW;                                                                          \
      if constexpr (std::is_same<TE, uint16_t>::value) {                                                                   \
_Pragma("unroll")                                                                                                          \
        for (int kk = 0; kk < KBE; kk += 16) {                                                                             \
          bf16x8 a[TI], b[TJ];                                                                                             \
_Pragma("unroll")                                                                                                          \
          for (int i = 0; i < TI; ++i)                                                                                     \
            a[i] = *reinterpret_cast<const bf16x8*>(&Asb[(i * 32 + (lane & 31)) * LDW + kk + (lane >> 5) * 8]);            \
_Pragma("unroll")                                                                                                          \
          for (int j = 0; j < TJ; ++j)                                                                                     \
            b[j] = *reinterpret_cast<const bf16x8*>(&Bsb[(j * 32 + (lane & 31)) * LDW + kk + (lane >> 5) * 8]);            \
_Pragma("unroll")                                                                                                          \
          for (int i = 0; i < TI; ++i)                                                                                     \
_Pragma("unroll")                                                                                                          \
            for (int j = 0; j < TJ; ++j)                                                                                   \
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0); \
        }                                                                                                                  \
        HTLR_PIPELINE(KBE / 16, TI + TJ, TI * TJ);                                                                         \
      } else if constexpr (std::is_same<TE, float>::value) {                                                               \
_Pragma("unroll")                                                                                                          \
        for (int kk = 0; kk < KBE; kk += 2) {                                                                              \
          float a[TI], b[TJ];                                                                                              \
_Pragma("unroll")                                                                                                          \
          for (int i = 0; i < TI; ++i) a[i] = Asb[(i * 32 + (lane & 31)) * LDW + kk + (lane >> 5)];                        \
_Pragma("unroll")                                                                                                          \
          for (int j = 0; j < TJ; ++j) b[j] = Bsb[(j * 32 + (lane & 31)) * LDW + kk + (lane >> 5)];                        \
_Pragma("unroll")                                                                                                          \
          for (int i = 0; i < TI; ++i)                                                                                     \
_Pragma("unroll")                                                                                                          \
            for (int j = 0; j < TJ; ++j)                                                                                   \
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);  \
        }                                                                                                                  \
        HTLR_PIPELINE(KBE / 2, TI + TJ, TI * TJ);                                                                          \
      } else {                                                                                                             \
_Pragma("unroll")                                                                                                          \
        for (int kk = 0; kk < KBE; kk += 4) {                                                                              \
          double a[TI], b[TJ];                                                                                             \
_Pragma("unroll")                                                                                                          \
          for (int i = 0; i < TI; ++i) a[i] = Asb[(i * 16 + (lane & 15)) * LDW + kcol(kk)];                                \
_Pragma("unroll")                                                                                                          \
          for (int j = 0; j < TJ; ++j) b[j] = Bsb[(j * 16 + (lane & 15)) * LDW + kcol(kk)];                                \
_Pragma("unroll")                                                                                                          \
          for (int i = 0; i < TI; ++i)                                                                                     \
_Pragma("unroll")                                                                                                          \
            for (int j = 0; j < TJ; ++j)                                                                                   \
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);  \
        }                                                                                                                  \
        HTLR_PIPELINE(KBE / 4, TI + TJ, TI * TJ);                                                                          \
      }                                                                                                                    \
  }
// One stage S held in LDS buffer CUR: (RAN, RBN) hold or receive stage
// S + 1, (RAF, RBF) receive stage S + 2 (prefetch depth 2).
#define HTLR_STEP(CUR, RAF, RBF, RAN, RBN, S)                       \
  {                                                                 \
    if constexpr (DL) {                                             \
      if ((S) + 1 < nstage) HTLR_DLOAD_NEXT((CUR) ^ 1);             \
      HTLR_COMPUTE(CUR);                                            \
      __builtin_amdgcn_s_waitcnt(0x0F70); /* vmcnt(0): LDS written */ \
      __syncthreads();                                              \
    } else {                                                        \
    if constexpr (PD == 2) {                                        \
      if ((S) + 2 < nstage) HTLR_LOAD_NEXT(RAF, RBF);               \
    } else {                                                        \
      if ((S) + 1 < nstage) HTLR_LOAD_NEXT(RAN, RBN);               \
    }                                                               \
    HTLR_COMPUTE(CUR);                                              \
    if ((S) + 1 < nstage) HTLR_SSTORE(RAN, RBN, (CUR) ^ 1);         \
    __syncthreads();                                                \
    }                                                               \
  }

  if (nstage > 0) {
    int64_t eL = e0;   // position (offset entry, K step) of the last stage loaded
    int ksL = 0;
    HTLR_SET_DELTA(e0);
    if constexpr (DL) {
      HTLR_DLOAD(0, 0);
      __builtin_amdgcn_s_waitcnt(0x0F70);
    } else {
      HTLR_GLOAD(ra0, rb0, 0);
      HTLR_SSTORE(ra0, rb0, 0);
    }
    if constexpr (PD == 2) {
      if (nstage > 1) HTLR_LOAD_NEXT(ra1, rb1);
    }
    __syncthreads();
    int64_t st = 0;
    if constexpr (PD == 2) {
      for (; st + 1 < nstage; st += 2) {
        HTLR_STEP(0, ra0, rb0, ra1, rb1, st);
        HTLR_STEP(1, ra1, rb1, ra0, rb0, st + 1);
      }
      if (st < nstage) HTLR_STEP(0, ra0, rb0, ra1, rb1, st);
    } else {
      // one register slot: stage s + 1 is loaded into it while s is computed
      for (; st + 1 < nstage; st += 2) {
        HTLR_STEP(0, ra1, rb1, ra0, rb0, st);
        HTLR_STEP(1, ra1, rb1, ra0, rb0, st + 1);
      }
      if (st < nstage) HTLR_STEP(0, ra1, rb1, ra0, rb0, st);
    }
  }
#undef HTLR_STEP
#undef HTLR_COMPUTE
#undef HTLR_LOAD_NEXT
#undef HTLR_DLOAD_NEXT
#undef HTLR_DLOAD
#undef HTLR_AS
#undef HTLR_BS
#undef HTLR_SET_DELTA
#undef HTLR_GLOAD
#undef HTLR_SSTORE

  // write the owned output tile
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int col = wn * WNC + j * TM + (lane & (TM - 1));
      const int b = col / nrhs, r = col % nrhs;
      const int t = (b < NB) ? tile_tau[(int64_t)tile * NB + b] : -1;
      if (t < 0) continue;
      // output slot: the target box, or (offset-major mode) the pair's partial buffer
      const int slot = tile_out ? tile_out[(int64_t)tile * NB + b] : t;
      TA* Ho = H + ((int64_t)slot * nrhs + r) * P;
      if constexpr (k16) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // f64 16x16x4 accumulator: register v holds row lane/16 + 4 v
          const int row = m0 + wm * WR + i * 16 + (lane >> 4) + 4 * v;
          if (row < P) Ho[row] = acc[i][j][v];
        }
      } else {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = m0 + wm * WR + i * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
          if (row < P) Ho[row] = acc[i][j][v];
        }
      }
    }
}

inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t m = 0;
  for (int b = 0; b < 21; ++b)
    m |= ((uint64_t)((x >> b) & 1) << (3 * b)) | ((uint64_t)((y >> b) & 1) << (3 * b + 1)) |
         ((uint64_t)((z >> b) & 1) << (3 * b + 2));
  return m;
}

}  // namespace

// Whether the matrix-core path serves this level of the matrix and precision.
bool core_mfma_ok(const htlr_matrix_impl& A, const LevelData& lv, int prec) {
  if (!A.uniform || lv.P < 64) return false;
  const int E = prec == HTLR_FP64 ? 2 : (prec == HTLR_FP32 ? 4 : 8);
  return lv.P % E == 0;
}

// Whether it serves at least one level.
bool core_mfma_any(const htlr_matrix_impl& A, int prec) {
  for (const LevelData& lv : A.levels)
    if (lv.npairs > 0 && core_mfma_ok(A, lv, prec)) return true;
  return false;
}

// Measured at 128^3 x 16 right-hand sides (level 4): tile-major items make
// the 64- and 32-bit core applies 4-5% faster (the row blocks of a tile read
// the same gathered sources together); the bfloat16 one is 3% slower.  Taking
// the tiles longest list first makes them another 3-4% faster (the launch
// ends on short boundary tiles instead of an uneven last round).
int core_item_order(const htlr_matrix_impl& A, int prec) {
  if (A.cur.order >= 0) return A.cur.order;
  return prec == HTLR_BF16_CORE ? 0 : 2;
}

// Work lists for tiles of nb boxes of one parity class, built on first use.
//
// A tile computes every offset of the union of its members' lists; a member
// for which an offset leaves the domain contributes a zero column there.
// Near the domain boundary the lists differ (at level 4 of a 16^3 grid only
// 27 of a class's 512 boxes have the full list), so the members of a tile
// are chosen in two passes.  Boxes with identical lists fill whole tiles in
// Morton order (no padding); the remaining boxes are grouped greedily: seed
// with the unassigned box with the longest list, then repeatedly add the box
// that adds the fewest offsets to the union (ties: longer list first, then
// Morton order).  On the 128^3 level-4 lists this cuts the padded work from
// 1.19x to 1.10x the useful work at 8 boxes per tile, and from 1.33x to
// 1.17x at 16 (level 3, where every box is near the boundary, stays at 1.48x
// at 8).  Tiles are then ordered by their first box's Morton code, so that
// consecutive tiles are spatial neighbours.
static LevelData::Tiles& tiles_for(htlr_matrix_impl& A, LevelData& lv, int nb) {
  for (auto& t : lv.tiles)
    if (t.nb == nb) return t;
  const int d = A.d, B = lv.B;
  const Csr& cs = lv.csr ? *lv.csr : A.plan.adm[lv.level];
  std::vector<int32_t> tau;
  std::vector<int64_t> ptr{0};
  std::vector<int4> off;
  // core id per offset, from the CSR entries of this level
  std::map<std::array<int, 3>, int> cid;
  for (int c = 0; c < lv.ncore; ++c)
    cid[{lv.offsets[3 * c], lv.offsets[3 * c + 1], lv.offsets[3 * c + 2]}] = c;
  const int words = (lv.ncore + 63) / 64;
  const int ncls = 1 << d;
  std::vector<int64_t> class_start{0};
  int64_t maxlist = 0;
  for (int cls = 0; cls < ncls; ++cls) {
    // boxes of the class, each with its offsets as a bit set over core ids
    std::vector<int32_t> boxes;
    for (int64_t t = 0; t < lv.nbox; ++t) {
      int x = (int)(t % B), y = (int)((t / B) % B), z = (int)(t / ((int64_t)B * B));
      int c = (x & 1) | ((y & 1) << 1) | (d == 3 ? ((z & 1) << 2) : 0);
      if (c == cls) boxes.push_back((int32_t)t);
    }
    const size_t nbx = boxes.size();
    std::vector<uint64_t> bits(nbx * words, 0);
    std::vector<int> len(nbx, 0);
    std::vector<uint64_t> mort(nbx);
    for (size_t q = 0; q < nbx; ++q) {
      const int64_t t = boxes[q];
      const int tx = (int)(t % B), ty = (int)((t / B) % B), tz = (int)(t / ((int64_t)B * B));
      mort[q] = morton3(tx >> 1, ty >> 1, tz >> 1);
      for (int64_t e = cs.ptr[t]; e < cs.ptr[t + 1]; ++e) {
        const int64_t sg = cs.src[e];
        const int c = cid.at({(int)(sg % B) - tx, (int)((sg / B) % B) - ty, (int)(sg / ((int64_t)B * B)) - tz});
        bits[q * words + c / 64] |= (uint64_t)1 << (c % 64);
      }
      len[q] = (int)(cs.ptr[t + 1] - cs.ptr[t]);
    }
    // boxes with identical lists first: full tiles in Morton order, no padding
    std::vector<size_t> order(nbx);
    for (size_t q = 0; q < nbx; ++q) order[q] = q;
    std::sort(order.begin(), order.end(), [&](size_t a, size_t b) {
      for (int w = 0; w < words; ++w)
        if (bits[a * words + w] != bits[b * words + w]) return bits[a * words + w] < bits[b * words + w];
      return mort[a] < mort[b];
    });
    std::vector<std::pair<uint64_t, std::vector<size_t>>> groups;
    std::vector<char> used(nbx, 0);
    size_t done = 0;
    for (size_t i = 0; i < nbx;) {
      size_t j = i + 1;
      while (j < nbx && std::equal(&bits[order[i] * words], &bits[order[i] * words] + words, &bits[order[j] * words]))
        ++j;
      for (size_t k = i; k + nb <= j; k += nb) {
        std::vector<size_t> g(order.begin() + k, order.begin() + k + nb);
        for (size_t q : g) used[q] = 1;
        done += nb;
        groups.push_back({mort[g[0]], g});
      }
      i = j;
    }
    // the rest greedily
    std::vector<uint64_t> uni(words);
    while (done < nbx) {
      size_t seed = nbx;
      for (size_t q = 0; q < nbx; ++q)
        if (!used[q] && (seed == nbx || len[q] > len[seed] || (len[q] == len[seed] && mort[q] < mort[seed]))) seed = q;
      std::vector<size_t> g{seed};
      used[seed] = 1;
      ++done;
      for (int w = 0; w < words; ++w) uni[w] = bits[seed * words + w];
      while ((int)g.size() < nb && done < nbx) {
        size_t best = nbx;
        int best_add = 0;
        for (size_t q = 0; q < nbx; ++q) {
          if (used[q]) continue;
          int add = 0;
          for (int w = 0; w < words; ++w) add += __builtin_popcountll(bits[q * words + w] & ~uni[w]);
          if (best == nbx || add < best_add || (add == best_add && (len[q] > len[best] ||
                                                                      (len[q] == len[best] && mort[q] < mort[best])))) {
            best = q;
            best_add = add;
          }
        }
        g.push_back(best);
        used[best] = 1;
        ++done;
        for (int w = 0; w < words; ++w) uni[w] |= bits[best * words + w];
      }
      groups.push_back({mort[seed], g});
    }
    std::stable_sort(groups.begin(), groups.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    // popularity of each offset: the number of the class's tiles whose list
    // holds it.  Every tile walks its offsets from the most to the least
    // popular, so the workgroups of one XCD, which run the class's tiles side
    // by side, read the same cores (A operand) at about the same time and
    // share them in L2; offsets only boundary tiles have come last.
    std::vector<int> pop(lv.ncore, 0);
    std::vector<std::vector<uint64_t>> unions;
    for (auto& gr : groups) {
      std::vector<uint64_t> u(words, 0);
      for (size_t q : gr.second)
        for (int w = 0; w < words; ++w) u[w] |= bits[q * words + w];
      for (int c = 0; c < lv.ncore; ++c)
        if (u[c / 64] >> (c % 64) & 1) ++pop[c];
      unions.push_back(std::move(u));
    }
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      auto& gr = groups[gi];
      const std::vector<uint64_t>& u = unions[gi];
      std::vector<std::pair<int, std::array<int, 3>>> ord;   // (-popularity, offset)
      for (int c = 0; c < lv.ncore; ++c)
        if (u[c / 64] >> (c % 64) & 1)
          ord.push_back({-pop[c], {lv.offsets[3 * c], lv.offsets[3 * c + 1], lv.offsets[3 * c + 2]}});
      std::sort(ord.begin(), ord.end());
      std::vector<std::array<int, 3>> offs;
      for (auto& po : ord) offs.push_back(po.second);
      // every member's own list must equal the tile list restricted to the domain
      for (size_t q : gr.second) {
        const int32_t t = boxes[q];
        int tx = t % B, ty = (t / B) % B, tz = t / (B * B);
        int64_t inside = 0;
        for (auto& o : offs) {
          int sx = tx + o[0], sy = ty + o[1], sz = tz + o[2];
          if (sx >= 0 && sx < B && sy >= 0 && sy < B && sz >= 0 && sz < B) ++inside;
        }
        if (inside != cs.ptr[t + 1] - cs.ptr[t])
          fail(HTLR_ERR_UNSUPPORTED, "admissible offsets differ inside a parity class");
      }
      for (int q = 0; q < nb; ++q) tau.push_back(q < (int)gr.second.size() ? boxes[gr.second[q]] : -1);
      for (auto& o : offs) off.push_back(make_int4(cid.at(o), o[0], o[1], o[2]));
      ptr.push_back((int64_t)off.size());
      maxlist = std::max<int64_t>(maxlist, (int64_t)offs.size());
    }
    class_start.push_back((int64_t)ptr.size() - 1);
  }
  lv.tiles.emplace_back();
  LevelData::Tiles& T = lv.tiles.back();
  T.nb = nb;
  T.ntile = (int64_t)ptr.size() - 1;
  T.class_start = class_start;
  T.maxlist = maxlist;
  for (size_t t = 0; t + 1 < ptr.size(); ++t) T.len.push_back(ptr[t + 1] - ptr[t]);
  T.tau.alloc(tau.size() * sizeof(int32_t));
  T.ptr.alloc(ptr.size() * sizeof(int64_t));
  T.off.alloc(std::max<size_t>(off.size(), 1) * sizeof(int4));
  HTLR_HIP(hipMemcpy(T.tau.ptr, tau.data(), tau.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HTLR_HIP(hipMemcpy(T.ptr.ptr, ptr.data(), ptr.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  if (!off.empty()) HTLR_HIP(hipMemcpy(T.off.ptr, off.data(), off.size() * sizeof(int4), hipMemcpyHostToDevice));
  A.device_bytes += T.tau.bytes + T.ptr.bytes + T.off.bytes;
  return T;
}

static int core_mfma_nb(int nrhs, int bnt) {
  int nb = 1;
  while (nb * 2 * nrhs <= bnt) nb *= 2;
  return nb;
}

// Tile shape for one level: 1 = 128x128, 2 = 128x64 (few columns), 3 = 256x128.
// 64-column tiles in FP64 take the 224-row shape when p^d fits it better
// than 128-row blocks do (192 < p^d <= 224).
// Cores of at most 64 rows (p^d <= 64, e.g. p = 4 in 3D, p = 8 in 2D) take
// 64-row tiles: 7 = 64x64, 6 = 64x128 (no padded half of a 128-row tile).
static int narrow_variant(const LevelData& lv, int prec) {
  if (lv.P <= 64) return 7;
  return (prec == HTLR_FP64 && lv.P > 192 && lv.P <= 224) ? 4 : 2;
}

static int pick_variant(const htlr_matrix_impl& A, const LevelData& lv, int nrhs, int prec) {
  if (A.cur.tile >= 1 && A.cur.tile <= 7) return A.cur.tile;
  const int64_t class_boxes = lv.nbox >> A.d;
  if (class_boxes * nrhs <= 64) return narrow_variant(lv, prec);
  if (lv.P <= 64) return 6;
  if (prec == HTLR_BF16_CORE && lv.P >= 256) return class_boxes * nrhs >= 256 ? 5 : 3;
  return 1;
}

// Tile shape of a variant: 1 = 128x128, 2 = 128x64, 3 = 256x128, 4 = 224x64
// (FP64; the other precisions run variant 4 as 128x64), 5 = 256x256
// (bfloat16, half the core reads per column; the others run it as 256x128),
// 6 = 64x128, 7 = 64x64.
static void variant_shape(int v, int prec, int* bmt, int* bnt) {
  *bmt = (v == 6 || v == 7) ? 64 : (v == 3 || v == 5) ? 256 : (v == 4 && prec == HTLR_FP64 ? 224 : 128);
  *bnt = (v == 2 || v == 4 || v == 7) ? 64 : (v == 5 && prec == HTLR_BF16_CORE ? 256 : 128);
}

template <typename TE> struct NarrowRows { static constexpr int value = 128; };
template <> struct NarrowRows<double> { static constexpr int value = 224; };
template <typename TE> struct WideCols { static constexpr int value = 128; };
template <> struct WideCols<uint16_t> { static constexpr int value = 256; };

// Sums the K-split partial results in a fixed order: H = sum_s part_s.
template <typename TA>
__global__ void k_reduce_parts(const TA* __restrict__ parts, TA* __restrict__ H, int64_t n, int ksplit,
                               int64_t stride) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    TA v = parts[i];
    for (int s = 1; s < ksplit; ++s) v += parts[s * stride + i];
    H[i] = v;
  }
}

// Number of K splits that gives the level enough workgroups: target > 0 is
// the tuner's choice of workgroups; 0 (automatic) aims for at least 2048 and
// at least 4 per unsplit work item.  Shorter workgroups balance the uneven
// offset lists of boundary tiles: at 128^3 x 16 (FP64, level 4: 2048 work
// items of about 500 offsets) 4 splits take the core apply from 324 to
// 296 ms; the partial sums add about 2 GB of traffic.
static int pick_ksplit(int64_t base_wgs, int64_t max_list, int target) {
  const int64_t tgt = target > 0 ? target : std::max<int64_t>(2048, 4 * base_wgs);
  int ks = 1;
  while (ks < 64 && base_wgs * ks < tgt && max_list / (ks * 2) >= 4) ks *= 2;
  return ks;
}

static LevelData::Tiles::Items& items_for(LevelData::Tiles& T, int ks, int nmb, int order, bool frozen) {
  const int key = ks + 64 * nmb + 4096 * order;
  auto it = T.items.find(key);
  if (it != T.items.end()) return it->second;
  if (frozen) fail(HTLR_ERR_INVALID, "matrix-core work list not reserved");
  // work items ordered (class, row block, split, tile) or (class, tile, row block, split);
  // order 2 takes each class's tiles from the longest offset list to the
  // shortest (ties in tile order), so that the launch ends on short items
  std::vector<int32_t> items;
  for (size_t cl = 0; cl + 1 < T.class_start.size(); ++cl) {
    if (order >= 1) {
      std::vector<int64_t> ts;
      for (int64_t t = T.class_start[cl]; t < T.class_start[cl + 1]; ++t) ts.push_back(t);
      if (order == 2)
        std::stable_sort(ts.begin(), ts.end(), [&](int64_t a, int64_t b) { return T.len[a] > T.len[b]; });
      for (int64_t t : ts)
        for (int mb = 0; mb < nmb; ++mb)
          for (int s = 0; s < ks; ++s) items.push_back((int32_t)((t << 12) | (mb << 6) | s));
    } else {
      for (int mb = 0; mb < nmb; ++mb)
        for (int s = 0; s < ks; ++s)
          for (int64_t t = T.class_start[cl]; t < T.class_start[cl + 1]; ++t)
            items.push_back((int32_t)((t << 12) | (mb << 6) | s));
    }
  }
  LevelData::Tiles::Items& I = T.items[key];
  I.buf.alloc(items.size() * sizeof(int32_t));
  HTLR_HIP(hipMemcpy(I.buf.ptr, items.data(), items.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  I.n = (int)items.size();
  return I;
}

template <typename TE, int BMT, int BNT>
static void launch_variant(const TE* G, const TE* W, const TE* zero, void* H, const int32_t* tau, const int64_t* ptr,
                           const int4* off, const LevelData::Tiles::Items& I, int ks, int64_t helems, int P, int nrhs,
                           int nb, int B, hipStream_t st) {
  using TA = typename AccT<TE>::type;
  const unsigned nwg = (unsigned)(((I.n + 7) / 8) * 8);
  hipLaunchKernelGGL((k_core_mfma<TE, BMT, BNT>), dim3(nwg), dim3(core_threads(BMT)), 0, st, G, W, zero, (TA*)H, tau,
                     ptr, off, I.buf.as<int32_t>(), I.n, ks, helems, P, nrhs, nb, B, (const int32_t*)nullptr);
}

template <typename TE, int BMT, int BNT>
static void launch_variant_out(const TE* G, const TE* W, const TE* zero, void* H, const LevelData::OffsetTiles& T,
                               int P, int nrhs, int B, hipStream_t st) {
  using TA = typename AccT<TE>::type;
  const unsigned nwg = (unsigned)(((T.nitems + 7) / 8) * 8);
  hipLaunchKernelGGL((k_core_mfma<TE, BMT, BNT>), dim3(nwg), dim3(core_threads(BMT)), 0, st, G, W, zero, (TA*)H,
                     T.tau.as<int32_t>(), T.ptr.as<int64_t>(), T.off.as<int4>(), T.items.as<int32_t>(), T.nitems, 1,
                     (int64_t)0, P, nrhs, T.nb, B, T.out.as<int32_t>());
}

// H_tau = sum of the partial products of tau's pairs, in a fixed order (the
// box's pairs occupy the consecutive slots rptr[tau] .. rptr[tau + 1] - 1).
template <typename TA>
__global__ void k_reduce_pairs(const TA* __restrict__ partial, TA* __restrict__ H, const int64_t* __restrict__ rptr,
                               int64_t per_box) {
  const int64_t tau = blockIdx.x;
  const int64_t k0 = rptr[tau], k1 = rptr[tau + 1];
  for (int64_t e = threadIdx.x; e < per_box; e += blockDim.x) {
    const TA* src = partial + k0 * per_box + e;
    const int64_t n = k1 - k0;
    TA v = TA(0);
    int64_t k = 0;
    for (; k + 4 <= n; k += 4) {
      const TA a0 = src[k * per_box], a1 = src[(k + 1) * per_box];
      const TA a2 = src[(k + 2) * per_box], a3 = src[(k + 3) * per_box];
      v += a0;
      v += a1;
      v += a2;
      v += a3;
    }
    for (; k < n; ++k) v += src[k * per_box];
    H[tau * per_box + e] = v;
  }
}

// Offset-major work lists: one group of tiles per offset, each tile holding
// boxes for which that offset is admissible, its columns' outputs going to
// per-pair slots.  A box's pairs take consecutive slots, in offset order.
static LevelData::OffsetTiles& offset_tiles_for(htlr_matrix_impl& A, LevelData& lv, int nb, int nmb, bool frozen) {
  for (auto& t : lv.otiles)
    if (t.nb == nb && t.nmb == nmb) return t;
  if (frozen) fail(HTLR_ERR_INVALID, "offset-major work list not reserved");
  const int B = lv.B;
  const Csr& cs = lv.csr ? *lv.csr : A.plan.adm[lv.level];
  std::map<std::array<int, 3>, int> cid;
  for (int c = 0; c < lv.ncore; ++c)
    cid[{lv.offsets[3 * c], lv.offsets[3 * c + 1], lv.offsets[3 * c + 2]}] = c;
  std::vector<std::vector<int32_t>> taus(lv.ncore);
  for (int64_t t = 0; t < lv.nbox; ++t) {
    const int tx = (int)(t % B), ty = (int)((t / B) % B), tz = (int)(t / ((int64_t)B * B));
    for (int64_t e = cs.ptr[t]; e < cs.ptr[t + 1]; ++e) {
      const int64_t sg = cs.src[e];
      const int c = cid.at({(int)(sg % B) - tx, (int)((sg / B) % B) - ty, (int)(sg / ((int64_t)B * B)) - tz});
      taus[c].push_back((int32_t)t);
    }
  }
  std::vector<int32_t> tau, out, items;
  std::vector<int64_t> ptr{0};
  std::vector<int4> off;
  std::vector<int64_t> rptr(lv.nbox + 1, 0);
  for (int c = 0; c < lv.ncore; ++c)
    for (int32_t t : taus[c]) ++rptr[t + 1];
  for (int64_t t = 0; t < lv.nbox; ++t) rptr[t + 1] += rptr[t];
  std::vector<int64_t> cursor(rptr.begin(), rptr.end() - 1);
  int64_t pair = 0;
  for (int c = 0; c < lv.ncore; ++c) {
    const int4 o = make_int4(c, lv.offsets[3 * c], lv.offsets[3 * c + 1], lv.offsets[3 * c + 2]);
    for (size_t s = 0; s < taus[c].size(); s += nb) {
      for (int q = 0; q < nb; ++q) {
        if (s + q < taus[c].size()) {
          const int32_t t = taus[c][s + q];
          tau.push_back(t);
          out.push_back((int32_t)cursor[t]++);
          ++pair;
        } else {
          tau.push_back(-1);
          out.push_back(-1);
        }
      }
      off.push_back(o);
      ptr.push_back((int64_t)off.size());
    }
  }
  const int64_t ntile = (int64_t)ptr.size() - 1;
  if (ntile >= (1 << 19)) fail(HTLR_ERR_UNSUPPORTED, "offset-major work list too large");
  if (pair >= ((int64_t)1 << 31)) fail(HTLR_ERR_UNSUPPORTED, "too many pairs for the offset-major mode");
  for (int64_t t = 0; t < ntile; ++t)
    for (int mb = 0; mb < nmb; ++mb) items.push_back((int32_t)((t << 12) | (mb << 6)));
  lv.otiles.emplace_back();
  LevelData::OffsetTiles& T = lv.otiles.back();
  T.nb = nb;
  T.nmb = nmb;
  T.npairs = pair;
  T.nitems = (int)items.size();
  auto up = [](DevBuf& b, const void* src, size_t bytes) {
    b.alloc(std::max<size_t>(bytes, 16));
    if (bytes) HTLR_HIP(hipMemcpy(b.ptr, src, bytes, hipMemcpyHostToDevice));
  };
  up(T.tau, tau.data(), tau.size() * sizeof(int32_t));
  up(T.out, out.data(), out.size() * sizeof(int32_t));
  up(T.ptr, ptr.data(), ptr.size() * sizeof(int64_t));
  up(T.off, off.data(), off.size() * sizeof(int4));
  up(T.items, items.data(), items.size() * sizeof(int32_t));
  up(T.rptr, rptr.data(), rptr.size() * sizeof(int64_t));
  A.device_bytes += T.tau.bytes + T.out.bytes + T.ptr.bytes + T.off.bytes + T.items.bytes + T.rptr.bytes;
  return T;
}

// Offset-major mode for a level: automatic when class tiles cannot fill
// their columns and the per-pair partial buffer stays modest.
static bool use_offset_major(const htlr_matrix_impl& A, const LevelData& lv, int nrhs, int prec) {
  const size_t esz = prec == HTLR_FP64 ? 8 : 4;
  const size_t partial = (size_t)lv.npairs * nrhs * lv.P * esz;
  if (A.cur.core_mode == 1) return false;
  if (A.cur.core_mode == 2) return partial <= ((size_t)1 << 31);
  const int64_t class_boxes = lv.nbox >> A.d;
  return class_boxes * nrhs < 128 && partial <= ((size_t)512 << 20);
}

// Tile shape of the offset-major mode: 128x64 unless an offset's boxes
// times right-hand sides fill well over 128 columns on average.
static int offset_major_variant(const htlr_matrix_impl& A, const LevelData& lv, int nrhs, int prec) {
  if (A.cur.tile >= 1 && A.cur.tile <= 7) return A.cur.tile;
  const int64_t avg = lv.npairs / std::max(lv.ncore, 1);
  return avg * nrhs <= 128 ? narrow_variant(lv, prec) : (lv.P <= 64 ? 6 : 1);
}

void launch_core_mfma(htlr_matrix_impl& A, LevelData& lv, int prec, const void* W, void* H, const void* zero,
                      int nrhs, hipStream_t st) {
  if ((int)A.ws.parts.size() <= lv.level) A.ws.parts.resize(lv.level + 1);
  if ((int)A.ws.pairs.size() <= lv.level) A.ws.pairs.resize(lv.level + 1);
  DevBuf& parts = A.ws.parts[lv.level];
  DevBuf& pairs = A.ws.pairs[lv.level];
  if (nrhs > kBNmax) fail(HTLR_ERR_UNSUPPORTED, "too many right-hand sides for the matrix-core tile");
  if (use_offset_major(A, lv, nrhs, prec)) {
    const int var = offset_major_variant(A, lv, nrhs, prec);
    int bmt, bnt;
    variant_shape(var, prec, &bmt, &bnt);
    const int nb = core_mfma_nb(nrhs, bnt);
    const int nmb = (lv.P + bmt - 1) / bmt;
    LevelData::OffsetTiles& T = offset_tiles_for(A, lv, nb, nmb, A.ws.frozen);
    const size_t esz = prec == HTLR_FP64 ? 8 : 4;
    const size_t need = (size_t)T.npairs * nrhs * lv.P * esz;
    if (pairs.bytes < need) {
      if (A.ws.frozen) fail(HTLR_ERR_INVALID, "pair buffer exceeds the reserved size");
      pairs.alloc(need);
    }
    void* Hp = pairs.ptr;
#define HTLR_LVO(TE, GPTR)                                                                                         \
  switch (var) {                                                                                                 \
    case 2: launch_variant_out<TE, 128, 64>(GPTR, (const TE*)W, (const TE*)zero, Hp, T, lv.P, nrhs, lv.B, st); break;   \
    case 4: launch_variant_out<TE, NarrowRows<TE>::value, 64>(GPTR, (const TE*)W, (const TE*)zero, Hp, T, lv.P, nrhs,  \
                                                             lv.B, st); break;                                       \
    case 5: launch_variant_out<TE, 256, WideCols<TE>::value>(GPTR, (const TE*)W, (const TE*)zero, Hp, T, lv.P, nrhs,   \
                                                            lv.B, st); break;                                        \
    case 3: launch_variant_out<TE, 256, 128>(GPTR, (const TE*)W, (const TE*)zero, Hp, T, lv.P, nrhs, lv.B, st); break;  \
    case 6: launch_variant_out<TE, 64, 128>(GPTR, (const TE*)W, (const TE*)zero, Hp, T, lv.P, nrhs, lv.B, st); break;   \
    case 7: launch_variant_out<TE, 64, 64>(GPTR, (const TE*)W, (const TE*)zero, Hp, T, lv.P, nrhs, lv.B, st); break;    \
    default: launch_variant_out<TE, 128, 128>(GPTR, (const TE*)W, (const TE*)zero, Hp, T, lv.P, nrhs, lv.B, st); break; \
  }
    if (prec == HTLR_BF16_CORE) {
      HTLR_LVO(uint16_t, lv.Gm16.as<uint16_t>());
    } else if (prec == HTLR_FP32) {
      HTLR_LVO(float, lv.Gm32.as<float>());
    } else {
      HTLR_LVO(double, lv.Gm64.as<double>());
    }
#undef HTLR_LVO
    HTLR_HIP(hipGetLastError());
    const int64_t per_box = (int64_t)nrhs * lv.P;
    if (prec == HTLR_FP64)
      hipLaunchKernelGGL(k_reduce_pairs<double>, dim3((unsigned)lv.nbox), dim3(256), 0, st, (const double*)Hp,
                         (double*)H, T.rptr.as<int64_t>(), per_box);
    else
      hipLaunchKernelGGL(k_reduce_pairs<float>, dim3((unsigned)lv.nbox), dim3(256), 0, st, (const float*)Hp,
                         (float*)H, T.rptr.as<int64_t>(), per_box);
    HTLR_HIP(hipGetLastError());
    return;
  }
  const int var = pick_variant(A, lv, nrhs, prec);
  int bmt, bnt;
  variant_shape(var, prec, &bmt, &bnt);
  const int nb = core_mfma_nb(nrhs, bnt);
  LevelData::Tiles& T = tiles_for(A, lv, nb);
  if (T.ntile == 0) return;
  const int nmb = (lv.P + bmt - 1) / bmt;
  const int ks = pick_ksplit(T.ntile * nmb, T.maxlist, A.cur.ks_target);
  if (T.ntile >= (1 << 19) || nmb > 63) fail(HTLR_ERR_UNSUPPORTED, "matrix-core work list too large");
  LevelData::Tiles::Items& I = items_for(T, ks, nmb, core_item_order(A, prec), A.ws.frozen);
  const size_t esz = prec == HTLR_FP64 ? 8 : 4;
  const int64_t helems = lv.nbox * (int64_t)nrhs * lv.P;
  void* Hout = H;
  if (ks > 1) {
    const size_t need = (size_t)helems * ks * esz;
    if (parts.bytes < need) {
      if (A.ws.frozen) fail(HTLR_ERR_INVALID, "K-split buffer exceeds the reserved size");
      parts.alloc(need);
    }
    Hout = parts.ptr;
  }
  const int32_t* tau = T.tau.as<int32_t>();
  const int64_t* ptr = T.ptr.as<int64_t>();
  const int4* off = T.off.as<int4>();
#define HTLR_LV(TE, GPTR)                                                                                          \
  switch (var) {                                                                                                 \
    case 2: launch_variant<TE, 128, 64>(GPTR, (const TE*)W, (const TE*)zero, Hout, tau, ptr, off, I, ks, helems,  \
                                        lv.P, nrhs, nb, lv.B, st); break;                                         \
    case 4: launch_variant<TE, NarrowRows<TE>::value, 64>(GPTR, (const TE*)W, (const TE*)zero, Hout, tau, ptr, off, I, ks, helems,  \
                                        lv.P, nrhs, nb, lv.B, st); break;                                         \
    case 5: launch_variant<TE, 256, WideCols<TE>::value>(GPTR, (const TE*)W, (const TE*)zero, Hout, tau, ptr, off, I, ks, helems,  \
                                        lv.P, nrhs, nb, lv.B, st); break;                                         \
    case 3: launch_variant<TE, 256, 128>(GPTR, (const TE*)W, (const TE*)zero, Hout, tau, ptr, off, I, ks, helems, \
                                         lv.P, nrhs, nb, lv.B, st); break;                                        \
    case 6: launch_variant<TE, 64, 128>(GPTR, (const TE*)W, (const TE*)zero, Hout, tau, ptr, off, I, ks, helems,  \
                                        lv.P, nrhs, nb, lv.B, st); break;                                         \
    case 7: launch_variant<TE, 64, 64>(GPTR, (const TE*)W, (const TE*)zero, Hout, tau, ptr, off, I, ks, helems,   \
                                       lv.P, nrhs, nb, lv.B, st); break;                                          \
    default: launch_variant<TE, 128, 128>(GPTR, (const TE*)W, (const TE*)zero, Hout, tau, ptr, off, I, ks,       \
                                          helems, lv.P, nrhs, nb, lv.B, st); break;                               \
  }
  if (prec == HTLR_BF16_CORE) {
    HTLR_LV(uint16_t, lv.Gm16.as<uint16_t>());
  } else if (prec == HTLR_FP32) {
    HTLR_LV(float, lv.Gm32.as<float>());
  } else {
    HTLR_LV(double, lv.Gm64.as<double>());
  }
#undef HTLR_LV
  HTLR_HIP(hipGetLastError());
  if (ks > 1) {
    const int blocks = (int)std::min<int64_t>((helems + 255) / 256, 4096);
    if (prec == HTLR_FP64)
      hipLaunchKernelGGL(k_reduce_parts<double>, dim3(blocks), dim3(256), 0, st, (const double*)parts.ptr, (double*)H,
                         helems, ks, helems);
    else
      hipLaunchKernelGGL(k_reduce_parts<float>, dim3(blocks), dim3(256), 0, st, (const float*)parts.ptr, (float*)H,
                         helems, ks, helems);
    HTLR_HIP(hipGetLastError());
  }
}

void reserve_workspace(htlr_matrix_impl& A, int nrhs) {
  A.ws.frozen = false;
  ensure_workspace(A, nrhs, HTLR_FP64);
  const int nl = A.L + 1;
  std::vector<size_t> parts_need(nl, 0), pairs_need(nl, 0);
  size_t nparts_need = 0;
  const TuneParams saved = A.cur;
  for (int c = 1; c <= nrhs; ++c) {
    for (int prec = 0; prec < 3; ++prec) {
      A.cur = find_tune(A, c, prec);
      if (use_near_leaves(A, c, prec, false))
        nparts_need = std::max(nparts_need, near_leaves_shape(A, c, prec, false).parts_bytes);
      if (!A.uniform) continue;
      const size_t esz = prec == HTLR_FP64 ? 8 : 4;
      for (LevelData& lv : A.levels) {
        if (lv.npairs == 0 || !core_mfma_ok(A, lv, HTLR_FP64)) continue;
        const int l = lv.level;
        if (use_offset_major(A, lv, c, prec)) {
          int bmt, bnt;
          variant_shape(offset_major_variant(A, lv, c, prec), prec, &bmt, &bnt);
          offset_tiles_for(A, lv, core_mfma_nb(c, bnt), (lv.P + bmt - 1) / bmt, false);
          pairs_need[l] = std::max(pairs_need[l], (size_t)lv.npairs * c * lv.P * esz);
          continue;
        }
        int bmt, bnt;
        variant_shape(pick_variant(A, lv, c, prec), prec, &bmt, &bnt);
        LevelData::Tiles& T = tiles_for(A, lv, core_mfma_nb(c, bnt));
        if (T.ntile == 0) continue;
        const int nmb = (lv.P + bmt - 1) / bmt;
        const int ks = pick_ksplit(T.ntile * nmb, T.maxlist, A.cur.ks_target);
        items_for(T, ks, nmb, core_item_order(A, prec), false);
        if (ks > 1) parts_need[l] = std::max(parts_need[l], (size_t)lv.nbox * c * lv.P * ks * esz);
      }
    }
  }
  A.cur = saved;
  if ((int)A.ws.parts.size() < nl) A.ws.parts.resize(nl);
  if ((int)A.ws.pairs.size() < nl) A.ws.pairs.resize(nl);
  for (int l = 0; l < nl; ++l) {
    if (A.ws.parts[l].bytes < parts_need[l]) A.ws.parts[l].alloc(parts_need[l]);
    if (A.ws.pairs[l].bytes < pairs_need[l]) A.ws.pairs[l].alloc(pairs_need[l]);
  }
  if (A.ws.nparts.bytes < nparts_need) A.ws.nparts.alloc(nparts_need);
  side_streams(A);
  A.ws.frozen = true;
}

// ---------------------------------------------------------------------------
// Near field on the matrix cores through the core apply.
//
// On a uniform grid with 8^3-point leaves the near-field block between a
// target leaf tau and a near leaf sigma (eq. 4.1 restricted to the pair)
// depends only on the offset Delta = sigma - tau: K_Delta[i][j] = T[|I - J|^2]
// with I and J the grid indices of target point i and source point j (T the
// distance table, whose entry 0 is the diagonal term of eq. 1.4).  So the
// near field is the same implicit GEMM as a level of the far field, with
// rows = the 512 target points, columns = (leaf, rhs) and K = (Delta, j),
// run by the class-tile kernel above on u gathered into leaf-major order.
// The block sums are the near kernels' sums in another order.

namespace {

constexpr int kLeafPts = 512;   // points of an 8^3 leaf, x fastest

__device__ __forceinline__ int64_t leaf_point(int leaf, int j, int n, int B) {
  const int lx = leaf % B, ly = (leaf / B) % B, lz = leaf / (B * B);
  return (int64_t)(lx * 8 + (j & 7)) + (int64_t)n * ((ly * 8 + ((j >> 3) & 7)) + (int64_t)n * (lz * 8 + (j >> 6)));
}

// K_Delta for every near offset: block (512^2 / 256, ncore), 256 threads.
template <typename T>
__global__ void k_near_block(const T* __restrict__ tab, const int4* __restrict__ off, T* __restrict__ G) {
  const int4 o = off[blockIdx.y];
  const int e = blockIdx.x * 256 + threadIdx.x;   // row i * 512 + column j
  const int i = e >> 9, j = e & 511;
  const int dx = (j & 7) + 8 * o.x - (i & 7);
  const int dy = ((j >> 3) & 7) + 8 * o.y - ((i >> 3) & 7);
  const int dz = (j >> 6) + 8 * o.z - (i >> 6);
  G[(int64_t)blockIdx.y * kLeafPts * kLeafPts + e] = tab[dx * dx + dy * dy + dz * dz];
}

// w[leaf][r][j] = u[r][point j of leaf]: block (leaf, r), 256 threads.
template <typename T>
__global__ void k_leaf_gather(const T* __restrict__ u, T* __restrict__ w, int n, int B, int nrhs) {
  const int leaf = blockIdx.x, r = blockIdx.y;
  const int64_t N = (int64_t)n * n * n;
  for (int j = threadIdx.x; j < kLeafPts; j += 256)
    w[((int64_t)leaf * nrhs + r) * kLeafPts + j] = u[(int64_t)r * N + leaf_point(leaf, j, n, B)];
}

// f[r][point i of leaf] = h[leaf][r][i] + a_i u[r][i]: block (leaf, r), 256 threads.
template <typename T>
__global__ void k_leaf_scatter(const T* __restrict__ h, const T* __restrict__ u, const T* __restrict__ a,
                               T* __restrict__ f, int n, int B, int nrhs) {
  const int leaf = blockIdx.x, r = blockIdx.y;
  const int64_t N = (int64_t)n * n * n;
  for (int i = threadIdx.x; i < kLeafPts; i += 256) {
    const int64_t g = leaf_point(leaf, i, n, B);
    const int64_t o = (int64_t)r * N + g;
    f[o] = h[((int64_t)leaf * nrhs + r) * kLeafPts + i] + a[g] * u[o];
  }
}

}  // namespace

bool near_tiles_ok(const htlr_matrix_impl& A, int nrhs) {
  return A.uniform && A.d == 3 && A.L >= 1 && A.plan.m[A.L] == 8 && A.kid != HTLR_K_POLY_TEST && A.Tsize > 0 &&
         nrhs >= 1 && nrhs <= kBNmax && !A.ws.frozen;
}

// The near level: distinct near offsets (host lists, built once) and their
// blocks in the precision asked for (each built on first use).
static void near_blocks(htlr_matrix_impl& A, LevelData& lv, bool f64);
static LevelData& near_level(htlr_matrix_impl& A, bool f64) {
  if (A.near_lv) {
    near_blocks(A, *A.near_lv, f64);
    return *A.near_lv;
  }
  const Plan& pl = A.plan;
  const Csr& cs = pl.near;
  auto nl = std::make_unique<LevelData>();
  LevelData& lv = *nl;
  lv.level = A.L + 1;
  lv.B = pl.B[A.L];
  lv.m = 8;
  lv.P = kLeafPts;
  lv.rank = 8;
  lv.nbox = A.levels[A.L].nbox;
  lv.npairs = cs.nnz();
  lv.csr = &cs;
  const int B = lv.B;
  std::map<std::array<int, 3>, int> cid;
  for (int64_t t = 0; t < lv.nbox; ++t)
    for (int64_t e = cs.ptr[t]; e < cs.ptr[t + 1]; ++e) {
      const int64_t sg = cs.src[e];
      const std::array<int, 3> o{(int)(sg % B) - (int)(t % B), (int)((sg / B) % B) - (int)((t / B) % B),
                                 (int)(sg / ((int64_t)B * B)) - (int)(t / ((int64_t)B * B))};
      if (cid.emplace(o, (int)cid.size()).second) lv.offsets.insert(lv.offsets.end(), o.begin(), o.end());
    }
  lv.ncore = (int)cid.size();
  if (lv.ncore == 0) fail(HTLR_ERR_UNSUPPORTED, "no near leaves");
  // every table index of a block must lie in the table
  for (int c = 0; c < lv.ncore; ++c) {
    int64_t d2 = 0;
    for (int k = 0; k < 3; ++k) {
      const int64_t dm = 8 * (int64_t)std::abs(lv.offsets[3 * c + k]) + 7;
      d2 += dm * dm;
    }
    if (d2 >= A.Tsize) fail(HTLR_ERR_UNSUPPORTED, "near block outside the distance table");
  }
  std::vector<int4> off(lv.ncore);
  for (int c = 0; c < lv.ncore; ++c)
    off[c] = make_int4(lv.offsets[3 * c], lv.offsets[3 * c + 1], lv.offsets[3 * c + 2], 0);
  A.near_off.alloc(off.size() * sizeof(int4));
  HTLR_HIP(hipMemcpy(A.near_off.ptr, off.data(), off.size() * sizeof(int4), hipMemcpyHostToDevice));
  A.near_zero.alloc(kLeafPts * sizeof(double));
  HTLR_HIP(hipMemset(A.near_zero.ptr, 0, A.near_zero.bytes));
  A.device_bytes += A.near_off.bytes + A.near_zero.bytes;
  A.near_lv = std::move(nl);
  near_blocks(A, *A.near_lv, f64);
  return *A.near_lv;
}

static void near_blocks(htlr_matrix_impl& A, LevelData& lv, bool f64) {
  DevBuf& G = f64 ? lv.Gm64 : lv.Gm32;
  if (G.ptr) return;
  const size_t blk = (size_t)lv.ncore * kLeafPts * kLeafPts;
  const dim3 grid(kLeafPts * kLeafPts / 256, lv.ncore);
  G.alloc(blk * (f64 ? sizeof(double) : sizeof(float)));
  if (f64)
    hipLaunchKernelGGL(k_near_block<double>, grid, dim3(256), 0, 0, A.T64.as<double>(), A.near_off.as<int4>(),
                       G.as<double>());
  else
    hipLaunchKernelGGL(k_near_block<float>, grid, dim3(256), 0, 0, A.T32.as<float>(), A.near_off.as<int4>(),
                       G.as<float>());
  HTLR_HIP(hipGetLastError());
  HTLR_HIP(hipDeviceSynchronize());
  A.device_bytes += G.bytes;
}

template <typename T>
void launch_near_tiles(htlr_matrix_impl& A, const T* u, T* f, int nrhs, hipStream_t st) {
  if (!near_tiles_ok(A, nrhs)) fail(HTLR_ERR_UNSUPPORTED, "near field on the core apply does not serve this product");
  const bool f64 = std::is_same<T, double>::value;
  LevelData& lv = near_level(A, f64);
  const size_t need = (size_t)lv.nbox * nrhs * kLeafPts * sizeof(T);
  if (A.near_w.bytes < need) {
    A.near_w.alloc(need);
    A.near_h.alloc(need);
  }
  const int n = A.n, B = lv.B;
  const T* a = f64 ? (const T*)A.a64.ptr : (const T*)A.a32.ptr;
  const dim3 grid((unsigned)lv.nbox, nrhs);
  hipLaunchKernelGGL(k_leaf_gather<T>, grid, dim3(256), 0, st, u, (T*)A.near_w.ptr, n, B, nrhs);
  HTLR_HIP(hipGetLastError());
  launch_core_mfma(A, lv, f64 ? HTLR_FP64 : HTLR_FP32, A.near_w.ptr, A.near_h.ptr, A.near_zero.ptr, nrhs, st);
  hipLaunchKernelGGL(k_leaf_scatter<T>, grid, dim3(256), 0, st, (const T*)A.near_h.ptr, u, a, f, n, B, nrhs);
  HTLR_HIP(hipGetLastError());
}

template void launch_near_tiles<double>(htlr_matrix_impl&, const double*, double*, int, hipStream_t);
template void launch_near_tiles<float>(htlr_matrix_impl&, const float*, float*, int, hipStream_t);

}  // namespace htlr
