// MFMA GEMM tile loop for gfx950 (included by the per-precision translation units).
//
//   C = alpha * sum_seg A_seg * B_seg + beta * X       (up to 2 summed K segments)
//
// Operand tiles are staged in LDS as [row][k] (k contiguous), double-buffered: while the waves
// run the MFMAs of tile t from one buffer, the global loads of tile t+1 are in flight and are
// written to the other buffer afterwards, so each K tile costs one barrier. k-contiguous
// operands are read with 16-byte (or wider) vector loads; the symmetric operators Hs, S and P are
// always read that way (P^T = P). Row strides are padded so that MFMA fragment reads hit
// distinct LDS banks.
//
// Modes:
//   CF64     v_mfma_f64_16x16x4f64   A, B fragments: lane l holds (row l%16, k l/16);
//                                     result rows l/16 + 4r, column l%16.
//   CF32     v_mfma_f32_16x16x4f32   same fragments; result rows 4(l/16) + r.
//   CBF16X3  v_mfma_f32_16x16x32_bf16 on a hi/lo split of each operand (a = hi + lo,
//            hi = bf16(a), lo = bf16(a - hi)); three products lo*hi + hi*lo + hi*hi per K step,
//            FP32 accumulation. Lane l holds row l%16, k 8(l/16)..8(l/16)+7; result rows
//            4(l/16) + r. Operands are either pre-split bf16 planes or FP32/FP64 values split
//            while a tile is staged.
//   CBF16X2A / CBF16X2B  the same with A (B) exactly representable in bf16: only its hi plane
//            is staged and two products remain (hi*lo + hi*hi).
//   CBF16X1  both operands single bf16 planes: one product hi*hi.
#pragma once

#include <type_traits>
#include <utility>

#include "omm_internal.h"

namespace omm {
namespace gemm_detail {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct GemmBatch {
  GemmOp op[4];
};

typedef void (*gemm_fn)(GemmBatch, const int*, int, double*);

__device__ __forceinline__ d4 mfma4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ T ldg(const void* p, int64_t i) {
  return static_cast<const T*>(p)[i];
}

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}

// Linear workgroup id -> (tm, tn): each of the 8 XCDs gets a contiguous run of tiles, M fastest,
// so tiles sharing a column panel of B are co-resident on one XCD (shared L2).
__device__ __forceinline__ bool tile_of(int tiles_m, int tiles_n, int& tm, int& tn) {
  const int total = tiles_m * tiles_n;
  const int per = (total + 7) >> 3;
  const int bid = blockIdx.x;
  const int t = (bid & 7) * per + (bid >> 3);
  if (t >= total) return false;
  tm = t % tiles_m;
  tn = t / tiles_m;
  return true;
}

// Tiles an op computes (bm x bn macro tiles): all of them, or for a symmetric (tri) op the
// tiles with tm <= tn. op_tile maps an index in [0, op_tiles) to (tm, tn): M fastest, and for
// a tri op column tn holds tm = 0 .. tn.
__host__ __device__ __forceinline__ int op_tiles(const GemmOp& op, int bm, int bn) {
  const int tm = (op.M + bm - 1) / bm, tn = (op.N + bn - 1) / bn;
  return op.tri ? tn * (tn + 1) / 2 : tm * tn;
}
__device__ __forceinline__ void op_tile(const GemmOp& op, int bm, int t, int& tm, int& tn) {
  if (op.tri) {
    int c = 0;
    while ((c + 1) * (c + 2) / 2 <= t) ++c;
    tn = c;
    tm = t - c * (c + 1) / 2;
  } else {
    const int tiles_m = (op.M + bm - 1) / bm;
    tm = t % tiles_m;
    tn = t / tiles_m;
  }
}

// K range [kb, ke) of segment `seg` owned by split `sp` (splits cut the concatenated K of all
// segments into BK-aligned chunks).
template <int BK>
__device__ __forceinline__ void split_range(const GemmOp& op, int seg, int sp, int nsplit, int& kb,
                                            int& ke) {
  const int ktot = op.K[0] + (op.nseg > 1 ? op.K[1] : 0);
  const int nk = (ktot + BK - 1) / BK;
  const int per = (nk + nsplit - 1) / nsplit;
  const int g0 = sp * per * BK, g1 = min(ktot, (sp + 1) * per * BK);
  const int off = seg == 0 ? 0 : op.K[0];
  kb = max(g0 - off, 0);
  ke = min(g1 - off, op.K[seg]);
}

// The part [g0, g1) of the concatenated K of all segments that falls in segment `seg`.
__device__ __forceinline__ void seg_range(const GemmOp& op, int seg, int g0, int g1, int& kb,
                                          int& ke) {
  const int off = seg == 0 ? 0 : op.K[0];
  kb = max(g0 - off, 0);
  ke = min(g1 - off, op.K[seg]);
}

// Per-mode element types: LDS element, register staging element, vector width of KC loads.
template <int MODE>
struct ModeTraits;
template <>
struct ModeTraits<CF64> {
  typedef double lds_t;
  static constexpr int VEC = 2;  // 16 B
  static constexpr int PAD = 2;
};
template <>
struct ModeTraits<CF32> {
  typedef float lds_t;
  static constexpr int VEC = 4;  // 16 B
  static constexpr int PAD = 4;
};
template <>
struct ModeTraits<CBF16X3> {
  typedef unsigned short lds_t;
  static constexpr int VEC = 8;  // 8 elements -> one 16-byte hi and one 16-byte lo LDS write
  static constexpr int PAD = 8;
};
template <>
struct ModeTraits<CBF16X2A> : ModeTraits<CBF16X3> {};
template <>
struct ModeTraits<CBF16X2B> : ModeTraits<CBF16X3> {};
template <>
struct ModeTraits<CBF16X1> : ModeTraits<CBF16X3> {};

// Global -> register staging of one operand tile (R rows x BK), `NV` vectors of VEC per thread.
// KC: vector = VEC consecutive k of one row. RC: vector = VEC consecutive rows of one k.
// TS = unsigned short means pre-split bf16 planes (hi at X, lo at Xlo), copied without conversion.
// LDS element offset of (row r, k). Padded rows, or (SWZ, BF16x3 with BK = 32) unpadded 64-byte
// rows whose four 16-byte chunks are rotated by r/2. A 16-byte-per-lane LDS read is served 16
// lanes per clock, lanes 8h .. 8h + 7 together with 8h + 16 .. 8h + 23: for a 16 x 16 fragment
// (lane % 16 = row, lane / 16 = chunk) those are 8 rows at two chunks, and the r/2 rotation puts
// them on 16 distinct 16-byte bank groups (a rotation by r/4 or r leaves them 2-way
// conflicted).
template <bool SWZ, int RS>
__device__ __forceinline__ int lds_off(int r, int k) {
  if constexpr (SWZ) return r * RS + ((((k >> 3) + (r >> 1)) & 3) << 3) + (k & 7);
  else return r * RS + k;
}

// ONE: the operand is a single bf16 plane (exact values): the lo plane is neither read nor
// staged.
template <int MODE, typename TS, int LAYOUT, int R, int BK, int NT, bool SWZ = false,
          bool ONE = false>
struct Stager {
  static constexpr int VEC = ModeTraits<MODE>::VEC;
  static constexpr int NV = R * BK / VEC / NT;
  static_assert(R * BK % (VEC * NT) == 0, "tile not divisible among threads");
  static constexpr bool PL = std::is_same<TS, unsigned short>::value;
  static_assert(!PL || is_bf16_mode(MODE), "bf16 planes feed the BF16x3 modes only");
  static_assert(!ONE || PL, "a single-plane operand is a bf16 plane");
  typedef typename ModeTraits<MODE>::lds_t lds_t;
  static_assert(!SWZ || (is_bf16_mode(MODE) && BK == 32), "swizzle: BF16x3 with BK = 32 only");
  static constexpr int RS = SWZ ? BK : BK + ModeTraits<MODE>::PAD;  // LDS row stride (elements)
  float rf[(MODE == CF64 || PL) ? 1 : NV * VEC];
  double rd[MODE == CF64 ? NV * VEC : 1];
  u16x8 ph[PL ? NV : 1], pq[PL && !ONE ? NV : 1];

  __device__ __forceinline__ void coords(int tid, int v, int& r, int& k) const {
    const int e = tid + v * NT;
    if (LAYOUT == KC) {
      r = e / (BK / VEC);
      k = (e % (BK / VEC)) * VEC;
    } else {
      k = e / (R / VEC);
      r = (e % (R / VEC)) * VEC;
    }
  }

  __device__ __forceinline__ void put(int idx, double v) {
    if constexpr (MODE == CF64) rd[idx] = v; else rf[idx] = (float)v;
  }

  // Whole tile in bounds with aligned rows: unconditional vector loads (one uniform branch per
  // tile instead of one per vector).
  __device__ __forceinline__ bool full_tile(int r0, int rmax, int k0, int ke, bool vec_ok) const {
    // uniform across the block: make it a scalar branch
    const int f = vec_ok && r0 + R <= rmax && k0 + BK <= ke;
    return __builtin_amdgcn_readfirstlane(f) != 0;
  }

  __device__ __forceinline__ void load_full(const void* X, const void* Xlo, int64_t ld, int r0, int k0,
                                            int tid) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      int r, k;
      coords(tid, v, r, k);
      const int gr = r0 + r, gk = k0 + k;
      const int64_t off = LAYOUT == KC ? (int64_t)gr * ld + gk : (int64_t)gk * ld + gr;
      if constexpr (PL) {
        ph[v] = *reinterpret_cast<const u16x8*>(static_cast<const unsigned short*>(X) + off);
        if constexpr (!ONE)
          pq[v] = *reinterpret_cast<const u16x8*>(static_cast<const unsigned short*>(Xlo) + off);
      } else if (LAYOUT == KC) {
        const TS* p = static_cast<const TS*>(X) + off;
        if constexpr (sizeof(TS) == 8) {
#pragma unroll
          for (int u = 0; u < VEC; u += 2) {
            const double2 q = *reinterpret_cast<const double2*>(p + u);
            put(v * VEC + u, q.x);
            put(v * VEC + u + 1, q.y);
          }
        } else {
#pragma unroll
          for (int u = 0; u < VEC; u += 4) {
            const float4 q = *reinterpret_cast<const float4*>(p + u);
            put(v * VEC + u, q.x);
            put(v * VEC + u + 1, q.y);
            put(v * VEC + u + 2, q.z);
            put(v * VEC + u + 3, q.w);
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < VEC; ++u) put(v * VEC + u, (double)ldg<TS>(X, off + u));
      }
    }
  }

  __device__ __forceinline__ void load(const void* X, const void* Xlo, int64_t ld, int r0, int rmax,
                                       int k0, int ke, int tid, bool vec_ok) {
    if (full_tile(r0, rmax, k0, ke, vec_ok)) {
      load_full(X, Xlo, ld, r0, k0, tid);
      return;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      int r, k;
      coords(tid, v, r, k);
      const int gr = r0 + r, gk = k0 + k;
      if constexpr (PL) {
        const unsigned short* hp = static_cast<const unsigned short*>(X);
        const unsigned short* lp = static_cast<const unsigned short*>(Xlo);
        if (LAYOUT == KC) {
          const int64_t off = (int64_t)gr * ld + gk;
          if (vec_ok && gr < rmax && gk + 8 <= ke) {
            ph[v] = *reinterpret_cast<const u16x8*>(hp + off);
            if constexpr (!ONE) pq[v] = *reinterpret_cast<const u16x8*>(lp + off);
          } else {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const bool in = gr < rmax && gk + u < ke;
              ph[v][u] = in ? hp[off + u] : (unsigned short)0;
              if constexpr (!ONE) pq[v][u] = in ? lp[off + u] : (unsigned short)0;
            }
          }
        } else {
          const int64_t off = (int64_t)gk * ld + gr;
          if (vec_ok && gk < ke && gr + 8 <= rmax) {
            ph[v] = *reinterpret_cast<const u16x8*>(hp + off);
            if constexpr (!ONE) pq[v] = *reinterpret_cast<const u16x8*>(lp + off);
          } else {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const bool in = gr + u < rmax && gk < ke;
              ph[v][u] = in ? hp[off + u] : (unsigned short)0;
              if constexpr (!ONE) pq[v][u] = in ? lp[off + u] : (unsigned short)0;
            }
          }
        }
      } else if (LAYOUT == KC) {
        const bool full = vec_ok && gr < rmax && gk + VEC <= ke;
        const TS* p = static_cast<const TS*>(X) + (int64_t)gr * ld + gk;
        if (full) {
          if constexpr (sizeof(TS) == 8) {
#pragma unroll
            for (int u = 0; u < VEC; u += 2) {
              const double2 q = *reinterpret_cast<const double2*>(p + u);
              put(v * VEC + u, q.x);
              put(v * VEC + u + 1, q.y);
            }
          } else {
#pragma unroll
            for (int u = 0; u < VEC; u += 4) {
              const float4 q = *reinterpret_cast<const float4*>(p + u);
              put(v * VEC + u, q.x);
              put(v * VEC + u + 1, q.y);
              put(v * VEC + u + 2, q.z);
              put(v * VEC + u + 3, q.w);
            }
          }
        } else {
#pragma unroll
          for (int u = 0; u < VEC; ++u)
            put(v * VEC + u, (gr < rmax && gk + u < ke) ? (double)p[u] : 0.0);
        }
      } else {
#pragma unroll
        for (int u = 0; u < VEC; ++u) {
          const bool in = gr + u < rmax && gk < ke;
          put(v * VEC + u, in ? (double)ldg<TS>(X, (int64_t)gk * ld + gr + u) : 0.0);
        }
      }
    }
  }

  // Registers -> LDS buffer(s) [R][RS]. BF16X3 writes hi to s0 and lo to s1.
  __device__ __forceinline__ void store(lds_t* s0, lds_t* s1, int tid) const {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      int r, k;
      coords(tid, v, r, k);
      if constexpr (PL) {
        if (LAYOUT == KC) {
          *reinterpret_cast<u16x8*>(s0 + lds_off<SWZ, RS>(r, k)) = ph[v];
          if constexpr (!ONE) *reinterpret_cast<u16x8*>(s1 + lds_off<SWZ, RS>(r, k)) = pq[v];
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            s0[lds_off<SWZ, RS>(r + u, k)] = ph[v][u];
            if constexpr (!ONE) s1[lds_off<SWZ, RS>(r + u, k)] = pq[v][u];
          }
        }
      } else if constexpr (is_bf16_mode(MODE)) {
        if (LAYOUT == KC) {
          u16x8 h, l;
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const float x = rf[v * VEC + u];
            const unsigned short hb = bf16_rne(x);
            h[u] = hb;
            l[u] = bf16_rne(x - bf16_val(hb));
          }
          *reinterpret_cast<u16x8*>(s0 + lds_off<SWZ, RS>(r, k)) = h;
          *reinterpret_cast<u16x8*>(s1 + lds_off<SWZ, RS>(r, k)) = l;
        } else {
#pragma unroll
          for (int u = 0; u < VEC; ++u) {
            const float x = rf[v * VEC + u];
            const unsigned short hb = bf16_rne(x);
            s0[lds_off<SWZ, RS>(r + u, k)] = hb;
            s1[lds_off<SWZ, RS>(r + u, k)] = bf16_rne(x - bf16_val(hb));
          }
        }
      } else if constexpr (MODE == CF64) {
        if (LAYOUT == KC) {
#pragma unroll
          for (int u = 0; u < VEC; u += 2)
            *reinterpret_cast<double2*>(s0 + r * RS + k + u) = double2{rd[v * VEC + u], rd[v * VEC + u + 1]};
        } else {
#pragma unroll
          for (int u = 0; u < VEC; ++u) s0[(r + u) * RS + k] = rd[v * VEC + u];
        }
      } else {
        if (LAYOUT == KC) {
#pragma unroll
          for (int u = 0; u < VEC; u += 4)
            *reinterpret_cast<float4*>(s0 + r * RS + k + u) =
                float4{rf[v * VEC + u], rf[v * VEC + u + 1], rf[v * VEC + u + 2], rf[v * VEC + u + 3]};
        } else {
#pragma unroll
          for (int u = 0; u < VEC; ++u) s0[(r + u) * RS + k] = rf[v * VEC + u];
        }
      }
    }
  }
};

template <int MODE>
struct AccT {
  typedef f4 type;
};
template <>
struct AccT<CF64> {
  typedef d4 type;
};

// Stores output element (row, col) and, if the op asks for them, its bf16 planes.
template <typename TC>
__device__ __forceinline__ void store_out(const GemmOp& op, int row, int col, double v) {
  const TC c = (TC)v;
  static_cast<TC*>(op.C)[(int64_t)row * op.ldc + col] = c;
  if (op.Chi) {
    const double w = (double)c;
    const unsigned short h = bf16_rne((float)w);
    const int64_t e = (int64_t)row * op.ldp + col;
    static_cast<unsigned short*>(op.Chi)[e] = h;
    if (op.Clo)  // null: the next product reads the hi plane alone
      static_cast<unsigned short*>(op.Clo)[e] = bf16_rne((float)(w - (double)bf16_val(h)));
  }
}

// Epilogue of one wave's TM x TN blocks at (r0, c0): C = alpha acc + beta X, or the FP64 split-K
// partial at ws[(sp * nops + z) * M * N + ...].
template <int MODE, typename TC, typename TX, int TM, int TN, typename acc_t>
__device__ __forceinline__ void store_acc(const GemmOp& op, const acc_t (&acc)[TM][TN], int r0,
                                          int c0, int lane, int sp, int nsplit, double* ws, int z,
                                          int nops) {
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = MODE == CF64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
        const int row = r0 + i * 16 + rr;
        const int col = c0 + j * 16 + (lane & 15);
        if (row < op.M && col < op.N) {
          const double s = (double)acc[i][j][r];
          if (nsplit > 1) {
            ws[((int64_t)sp * nops + z) * op.M * op.N + (int64_t)row * op.N + col] = s;
          } else {
            double v = op.alpha * s;
            if (op.X) v += op.beta * (double)ldg<TX>(op.X, (int64_t)row * op.ldx + col);
            store_out<TC>(op, row, col, v);
          }
        }
      }
}

// One output tile (tm, tn) of op, K split `sp` of `nsplit`. WM x WN waves, each wave TM x TN
// blocks of 16 x 16; BK = K tile. Split-K partials go to ws[(sp * nops + z) * M * N + ...].
template <int MODE, typename TA, typename TB, typename TC, typename TX, int LA, int LB, int WM,
          int WN, int TM, int TN, int BK, bool SWZ = false>
__device__ __forceinline__ void gemm_tile(const GemmOp& op, int tm, int tn, int sp, int nsplit,
                                          double* ws, int z, int nops) {
  constexpr int NT = WM * WN * 64;
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16;
  constexpr bool ONE_A = one_plane_a(MODE), ONE_B = one_plane_b(MODE);
  typedef Stager<MODE, TA, LA, BM, BK, NT, SWZ, ONE_A> SA;
  typedef Stager<MODE, TB, LB, BN, BK, NT, SWZ, ONE_B> SB;
  typedef typename ModeTraits<MODE>::lds_t lds_t;
  constexpr int RS = SA::RS;
  // LDS planes per operand: hi + lo, or hi alone for a single-plane operand
  constexpr int NBA = is_bf16_mode(MODE) && !ONE_A ? 2 : 1;
  constexpr int NBB = is_bf16_mode(MODE) && !ONE_B ? 2 : 1;
  typedef typename AccT<MODE>::type acc_t;

  const int m0 = tm * BM, n0 = tn * BN;

  __shared__ __attribute__((aligned(16))) lds_t As[2][NBA][BM * RS];
  __shared__ __attribute__((aligned(16))) lds_t Bs[2][NBB][BN * RS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  SA sa;
  SB sb;
  for (int seg = 0; seg < op.nseg; ++seg) {
    int kb, ke;
    split_range<BK>(op, seg, sp, nsplit, kb, ke);
    if (kb >= ke) continue;
    const void* A = op.A[seg];
    const void* B = op.B[seg];
    const void* Al = op.Alo[seg];
    const void* Bl = op.Blo[seg];
    const int64_t lda = op.lda[seg], ldb = op.ldb[seg];
    const bool va = (SA::PL || LA == KC) && (lda % SA::VEC) == 0 &&
                    ((reinterpret_cast<uintptr_t>(A) & 15) == 0) &&
                    (!SA::PL || (reinterpret_cast<uintptr_t>(Al) & 15) == 0);
    const bool vb = (SB::PL || LB == KC) && (ldb % SB::VEC) == 0 &&
                    ((reinterpret_cast<uintptr_t>(B) & 15) == 0) &&
                    (!SB::PL || (reinterpret_cast<uintptr_t>(Bl) & 15) == 0);
    // K steps: kb, kb + BK, ... ; block-sparse B (one segment, no split): the BK-deep parts of
    // the listed 32-deep K blocks of the 256-column tile that holds this tile's columns (a step
    // past K loads zeros)
    constexpr int SUB = SPARSE_BK >= BK ? SPARSE_BK / BK : 1;
    const bool sparse = op.kptr != nullptr;
    const int lt = n0 / SPARSE_BN;  // list tile
    const int* kl = sparse ? op.kidx + op.kptr[lt] : nullptr;
    const int nsteps = sparse ? __builtin_amdgcn_readfirstlane(op.kptr[lt + 1] - op.kptr[lt]) * SUB
                              : (ke - kb + BK - 1) / BK;
    auto kstep = [&](int i) {
      return sparse ? __builtin_amdgcn_readfirstlane(kl[i / SUB]) * SPARSE_BK + (i % SUB) * BK
                    : kb + i * BK;
    };
    if (nsteps == 0) continue;
    __syncthreads();  // previous segment's readers are done with the buffers
    sa.load(A, Al, lda, m0, op.M, kstep(0), ke, tid, va);
    sb.load(B, Bl, ldb, n0, op.N, kstep(0), ke, tid, vb);
    sa.store(As[0][0], As[0][NBA - 1], tid);
    sb.store(Bs[0][0], Bs[0][NBB - 1], tid);
    __syncthreads();
    int buf = 0;
    for (int step = 0; step < nsteps; ++step) {
      const bool more = step + 1 < nsteps;
      if (more) {
        const int kn = kstep(step + 1);
        sa.load(A, Al, lda, m0, op.M, kn, ke, tid, va);
        sb.load(B, Bl, ldb, n0, op.N, kn, ke, tid, vb);
      }
      const lds_t* a0 = As[buf][0];
      const lds_t* b0 = Bs[buf][0];
      if constexpr (is_bf16_mode(MODE)) {
        const lds_t* a1 = As[buf][NBA - 1];
        const lds_t* b1 = Bs[buf][NBB - 1];
        // lo*hi terms first, hi*hi last (smaller terms enter the FP32 accumulator first)
        auto prod = [&](const bf8& ah, const bf8& al, const bf8& bh, const bf8& bl, f4 c) {
          if constexpr (!ONE_A)
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
          if constexpr (!ONE_B)
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
          return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
        };
        const int kof = 8 * (lane >> 4);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 32) {
          auto frag = [&](const lds_t* base, int r) {
            return __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(
                                               base + lds_off<SWZ, RS>(r, kk + kof)));
          };
          if constexpr (TM > TN) {
            // all B fragments live, one A pair at a time (fewer registers for tall wave tiles)
            bf8 bh[TN], bl[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              const int r = wn * TN * 16 + j * 16 + (lane & 15);
              bh[j] = frag(b0, r);
              bl[j] = ONE_B ? bh[j] : frag(b1, r);
            }
#pragma unroll
            for (int i = 0; i < TM; ++i) {
              const int r = wm * TM * 16 + i * 16 + (lane & 15);
              const bf8 ah = frag(a0, r), al = ONE_A ? ah : frag(a1, r);
#pragma unroll
              for (int j = 0; j < TN; ++j) acc[i][j] = prod(ah, al, bh[j], bl[j], acc[i][j]);
            }
          } else {
            bf8 ah[TM], al[TM];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
              const int r = wm * TM * 16 + i * 16 + (lane & 15);
              ah[i] = frag(a0, r);
              al[i] = ONE_A ? ah[i] : frag(a1, r);
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              const int r = wn * TN * 16 + j * 16 + (lane & 15);
              const bf8 bh = frag(b0, r), bl = ONE_B ? bh : frag(b1, r);
#pragma unroll
              for (int i = 0; i < TM; ++i) acc[i][j] = prod(ah[i], al[i], bh, bl, acc[i][j]);
            }
          }
        }
      } else {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
          const int kr = kk + (lane >> 4);
          lds_t a[TM], b[TN];
#pragma unroll
          for (int i = 0; i < TM; ++i) a[i] = a0[(wm * TM * 16 + i * 16 + (lane & 15)) * RS + kr];
#pragma unroll
          for (int j = 0; j < TN; ++j) b[j] = b0[(wn * TN * 16 + j * 16 + (lane & 15)) * RS + kr];
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = mfma4(a[i], b[j], acc[i][j]);
        }
      }
      if (more) {
        sa.store(As[buf ^ 1][0], As[buf ^ 1][NBA - 1], tid);
        sb.store(Bs[buf ^ 1][0], Bs[buf ^ 1][NBB - 1], tid);
      }
      __syncthreads();
      buf ^= 1;
    }
  }

  store_acc<MODE, TC, TX, TM, TN>(op, acc, m0 + wm * TM * 16, n0 + wn * TN * 16, lane, sp, nsplit,
                                  ws, z, nops);
}

// ---- direct-to-LDS pipeline: bf16 planes, A and B k-contiguous, 256 x 256 tile, 8 waves -----
// Full K stages go from memory straight into LDS (buffer_load_dwordx4 ... lds: lane l of a wave
// writes its 16 bytes at the wave's LDS base + 16 l), so no VGPRs hold staged tiles and no
// ds_write is issued. NS stage buffers rotate: the loads of stage t + NS - 1 are issued during
// stage t, which gives each load up to NS - 1 compute phases to land. The rotated-chunk row
// layout of the register path is kept: LDS slot (row r, chunk l % 4) receives logical chunk
// (l % 4 - l / 8) & 3 of row r (r = 16 j + l / 4, so (r / 2) % 4 = (l / 8) % 4). Rows past the
// matrix edge re-read the last row (their outputs are never stored); a stage that runs past the
// end of K takes the register path (zero fill). Requires 16-byte aligned plane pointers, leading
// dimensions that are multiples of 8, and a first segment length that is a multiple of 8
// (checked by the launcher). The loads take the buffer form rather than the global one: the
// compiler counts a global load into LDS as both a memory and an LDS operation, and after one
// it can only wait for all outstanding LDS reads at once, so every K step would wait for its
// whole first batch of fragment reads before its first MFMA. With the buffer form its LDS waits
// stay per read; the descriptor's record count (the plane's size) also bounds every load.
constexpr int DMA_BM = 256, DMA_BN = 256, DMA_BK = 32, DMA_PLANE = DMA_BM * DMA_BK;

// f(std::integral_constant<int, i>) for i = 0 .. N - 1, each i a compile-time constant
template <typename F, int... I>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}
// Loads i = 0 .. n - 1 spread over `span` slots: load i goes after slot i span / n.
constexpr int loads_in_slot(int g, int n, int span) {
  int c = 0;
  for (int i = 0; i < n; ++i) c += i * span / n == g;
  return c;
}
constexpr bool slots_cover(int n, int span) {  // every load lands in exactly one slot < span
  int c = 0;
  for (int g = 0; g < span; ++g) c += loads_in_slot(g, n, span);
  return c == n;
}
static_assert(slots_cover(4, 8) && slots_cover(6, 8) && slots_cover(8, 8) && slots_cover(8, 4),
              "one-, two- and three-product stages (4, 6, 8 wave loads over 8 or 4 groups)");
static_assert(DMA_BN == SPARSE_BN && DMA_BK == SPARSE_BK, "block-sparse lists follow this tile");
static_assert(DMA_BM == DMA_BN, "op_tiles / op_tile enumerate symmetric products on square tiles");

// s_waitcnt: vmcnt <= n, lgkmcnt = 0 (expcnt unconstrained)
template <int N>
__device__ __forceinline__ void wait_vm_lgkm0() {
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (0 << 8) | (((N >> 4) & 3) << 14));
}

constexpr int DMA_TM = 8, DMA_TN = 4;  // 16 x 16 blocks per wave (wave grid 2 x 4)
// LDS stages of the direct-to-LDS tile: 64 KB each with three products, 48 KB with two, 32 KB
// with one, in 160 KB
constexpr int dma_stages(int mode) {
  return mode == CBF16X3 ? 2 : mode == CBF16X1 ? 4 : 3;
}
template <int KIND, typename TC, typename TX>
struct DmaUser {
  static constexpr int kind = KIND;  // 0: one tile per workgroup, 1: stream-K
};

// Accumulates the K range [g0, g1) (concatenated over the segments) of tile (tm, tn) into acc.
// USER (the calling kernel and its output type) only makes each kernel instantiate its own copy:
// the host pass of hipcc rejects one such device template shared by two kernels.
template <int MODE, int NS, typename USER>
__device__ __forceinline__ void gemm_tile_dma_acc(const GemmOp& op, int tm, int tn, int g0, int g1,
                                                  f4 (&acc)[DMA_TM][DMA_TN]) {
  constexpr int WM = 2, TM = DMA_TM, TN = DMA_TN, NT = 512, BK = DMA_BK, RS = DMA_BK;
  constexpr bool ONE_A = one_plane_a(MODE), ONE_B = one_plane_b(MODE);
  constexpr int NBA = ONE_A ? 1 : 2, NBB = ONE_B ? 1 : 2, NPL = NBA + NBB;
  constexpr int NPROD = (ONE_A && ONE_B) ? 1 : (ONE_A || ONE_B) ? 2 : 3;
  constexpr int DPS = NPL * (DMA_BM * BK * 2 / 1024) / 8;  // 1 KB wave loads per wave per stage
  static_assert(is_bf16_mode(MODE), "direct-to-LDS path: bf16 planes only");
  static_assert(NS * NPL * DMA_PLANE * 2 + SPARSE_KL_MAX * 4 <= 160 * 1024, "LDS budget");
  typedef unsigned short lds_t;
  typedef Stager<MODE, unsigned short, KC, DMA_BM, BK, NT, true, ONE_A> SA;
  typedef Stager<MODE, unsigned short, KC, DMA_BN, BK, NT, true, ONE_B> SB;

  // Stage buffers, then the column tile's K-block list (block-sparse B), read from LDS: a global
  // load of the next entry would make every stage wait for all of its operand loads in flight.
  // One LDS object: with a second one the compiler makes every fragment read after a
  // direct-to-LDS load wait for that load.
  __shared__ __attribute__((aligned(16))) lds_t L[NS * NPL * DMA_PLANE + 2 * SPARSE_KL_MAX];
  int* const KL = reinterpret_cast<int*>(L + NS * NPL * DMA_PLANE);

  const int m0 = tm * DMA_BM, n0 = tn * DMA_BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0, 0, 0, 0};

  // this lane's row within a 16-row wave chunk, and the logical 8-element chunk it fetches
  const int lrow = lane >> 2, lchunk = ((lane & 3) - (lane >> 3)) & 3;

  for (int seg = 0; seg < op.nseg; ++seg) {
    int kb, ke;
    seg_range(op, seg, g0, g1, kb, ke);
    if (kb >= ke) continue;
    const unsigned short* plane[4];
    int64_t ldp[4];
    int row0[4], rmax[4];
    __amdgpu_buffer_rsrc_t rs[4];
    {
      int p = 0;
      plane[p] = static_cast<const unsigned short*>(op.A[seg]);
      ldp[p] = op.lda[seg]; row0[p] = m0; rmax[p] = op.M; ++p;
      if constexpr (!ONE_A) {
        plane[p] = static_cast<const unsigned short*>(op.Alo[seg]);
        ldp[p] = op.lda[seg]; row0[p] = m0; rmax[p] = op.M; ++p;
      }
      plane[p] = static_cast<const unsigned short*>(op.B[seg]);
      ldp[p] = op.ldb[seg]; row0[p] = n0; rmax[p] = op.N; ++p;
      if constexpr (!ONE_B) {
        plane[p] = static_cast<const unsigned short*>(op.Blo[seg]);
        ldp[p] = op.ldb[seg]; row0[p] = n0; rmax[p] = op.N; ++p;
      }
    }
    // raw buffer descriptors (stride 0, records = the plane's bytes, gfx9 default format word)
#pragma unroll
    for (int p = 0; p < NPL; ++p)
      rs[p] = __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned short*>(plane[p]), (short)0,
                                                (int)(unsigned)(2 * (int64_t)rmax[p] * ldp[p]),
                                                0x00020000);
    // per-lane byte offset (32 bits: the plane base stays a wave-uniform scalar) of each of
    // this wave's DPS wave loads; the k offset is added per stage. Wave chunk q = wave + 8 i
    // covers plane q / 16 = i / 2 (8 waves), rows 16 (q % 16) ..
    static_assert(NT == 512, "eight waves: wave chunk i lies in plane i / 2");
    unsigned off[DPS];
    int dst[DPS];  // LDS element offset within a stage buffer (wave-uniform)
#pragma unroll
    for (int i = 0; i < DPS; ++i) {
      const int pl = i >> 1, j = wave + 8 * (i & 1);
      const int gr = min(row0[pl] + 16 * j + lrow, rmax[pl] - 1);
      off[i] = (unsigned)(2 * ((int64_t)gr * ldp[pl] + 8 * lchunk));  // bytes
      dst[i] = pl * DMA_PLANE + 512 * j;
    }
    // dense: stages kb, kb + BK, ...; block-sparse B: the listed K blocks of this column tile
    const bool sparse = op.kptr != nullptr && op.nseg == 1;
    const int nst = sparse ? __builtin_amdgcn_readfirstlane(op.kptr[tn + 1] - op.kptr[tn])
                           : (ke - kb + BK - 1) / BK;
    // K offset of stage st and whether the stage is whole, both wave-uniform (the list entry is
    // read from LDS into a scalar; only the last stage can be partial)
    auto kstart = [&](int st) {
      return sparse ? __builtin_amdgcn_readfirstlane(KL[st]) * BK : kb + st * BK;
    };
    bool last_full = true;
    auto full = [&](int st) { return st + 1 < nst || last_full; };
    auto issue = [&](int st) {
      lds_t* buf = L + (st % NS) * NPL * DMA_PLANE;
      const int k0 = kstart(st);
      if (full(st)) {
#pragma unroll
        for (int i = 0; i < DPS; ++i)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rs[i >> 1], buf + dst[i], 16,
                                                   off[i] + 2u * (unsigned)k0, 0, 0, 0);
      } else {
        SA sa;
        SB sb;
        sa.load(op.A[seg], op.Alo[seg], op.lda[seg], m0, op.M, k0, ke, tid, true);
        sb.load(op.B[seg], op.Blo[seg], op.ldb[seg], n0, op.N, k0, ke, tid, true);
        sa.store(buf, buf + (NBA - 1) * DMA_PLANE, tid);
        sb.store(buf + NBA * DMA_PLANE, buf + (NPL - 1) * DMA_PLANE, tid);
      }
    };
    __syncthreads();  // the previous segment's readers are done with every buffer
    if (sparse) {  // nst <= ceil(K / 32) <= SPARSE_KL_MAX (checked by the launcher)
      const int* klist = op.kidx + op.kptr[tn];
      for (int e = tid; e < nst; e += NT) KL[e] = klist[e];
      __syncthreads();
    }
    if (nst > 0) last_full = kstart(nst - 1) + BK <= ke;
#pragma unroll
    for (int st = 0; st < NS - 1; ++st)
      if (st < nst) issue(st);
    // One stage. The direct-to-LDS loads of stage t + NS - 1 go into the buffer read in stage
    // t - 1. With SPREAD they are spread between this stage's MFMA groups, so that no wave
    // stalls issuing all of them at once while the memory pipeline drains; otherwise they (or
    // the register path of a partial stage) are issued before the compute.
    auto run_stage = [&](int t, auto spread_tag) {
      constexpr bool SPREAD = decltype(spread_tag)::value;
      // this wave's loads of stage t have landed (those of the issued stages after it, up to
      // t + NS - 2, may still be in flight), then every wave's have
      if (NS > 3 && t + 2 < nst && full(t + 2)) wait_vm_lgkm0<(NS > 3 ? 2 * DPS : 0)>();
      else if (NS > 2 && t + 1 < nst && full(t + 1)) wait_vm_lgkm0<(NS > 2 ? DPS : 0)>();
      else wait_vm_lgkm0<0>();
      __builtin_amdgcn_s_barrier();
      const int tnext = t + NS - 1;
      if (!SPREAD && tnext < nst) issue(tnext);
      const lds_t* buf = L + (t % NS) * NPL * DMA_PLANE;
      const lds_t* a0 = buf;
      const lds_t* a1 = buf + (NBA - 1) * DMA_PLANE;
      const lds_t* b0 = buf + NBA * DMA_PLANE;
      const lds_t* b1 = buf + (NPL - 1) * DMA_PLANE;
      const int kof = 8 * (lane >> 4);
      auto frag = [&](const lds_t* base, int r) {
        return __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(
                                           base + lds_off<true, RS>(r, kof)));
      };
      // Software pipeline over pairs of 16-row blocks: the A fragments of pair p + 1 are read
      // from LDS while the MFMAs of pair p run, so a wave waits on LDS once per stage (for its
      // B fragments and first pair) instead of once per pair.
      constexpr int PAIR = 2, NPAIR = TM / PAIR, NAR = ONE_A ? 1 : 2;
      constexpr int NBR = TN * (ONE_B ? 1 : 2);
      static_assert(TM % PAIR == 0, "row blocks come in pairs");
      bf8 ah[2][PAIR], al[2][PAIR], bh[TN], bl[TN];
      auto load_pair = [&](int p) {
#pragma unroll
        for (int q = 0; q < PAIR; ++q) {
          const int r = wm * TM * 16 + (p * PAIR + q) * 16 + (lane & 15);
          ah[p & 1][q] = frag(a0, r);
          al[p & 1][q] = ONE_A ? ah[p & 1][q] : frag(a1, r);
        }
      };
      auto mfma_row = [&](int p, int q) {
        const int i = p * PAIR + q;
        const bf8 h = ah[p & 1][q], l = al[p & 1][q];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          if constexpr (!ONE_A)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(l, bh[j], acc[i][j], 0, 0, 0);
          if constexpr (!ONE_B)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, bh[j], acc[i][j], 0, 0, 0);
        }
      };
      auto load_b = [&]() {
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int r = wn * TN * 16 + j * 16 + (lane & 15);
          bh[j] = frag(b0, r);
          bl[j] = ONE_B ? bh[j] : frag(b1, r);
        }
      };
      // MFMA group g (0 .. 2 NPAIR - 1) is followed by the stage-tnext loads i with
      // slot(i) = g: spread over all groups with three stages (a load has the rest of this
      // stage and the whole next one to land), over the first half with two (the rest of this
      // stage only).
      constexpr int NGRP = 2 * NPAIR, SPAN = NS > 2 ? NGRP : NGRP / 2;
      auto slot = [](int i) { return i * SPAN / DPS; };  // == loads_in_slot's rule
      auto pipelined = [&](auto with_loads) {
        constexpr bool WL = decltype(with_loads)::value;
        lds_t* nb = L + (tnext % NS) * NPL * DMA_PLANE;
        const unsigned kb2 = 2u * (unsigned)kstart(tnext);
        auto loads_after = [&](int g) {
          if constexpr (WL) {
#pragma unroll
            for (int i = 0; i < DPS; ++i)
              if (slot(i) == g)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs[i >> 1], nb + dst[i], 16,
                                                         off[i] + kb2, 0, 0, 0);
          }
        };
        load_pair(0);
        load_b();
#pragma unroll
        for (int p = 0; p < NPAIR; ++p) {
          mfma_row(p, 0);
          loads_after(2 * p);
          if (p + 1 < NPAIR) load_pair(p + 1);
          mfma_row(p, 1);
          loads_after(2 * p + 1);
        }
        // instruction groups for the scheduler: [reads of pair 0 and B] then, per pair p,
        // [MFMAs of its first row block] [its loads] [reads of pair p + 1] [MFMAs of its second
        // row block] [its loads]
        __builtin_amdgcn_sched_group_barrier(0x100, PAIR * NAR + NBR, 0);
        static_for<NPAIR>([&](auto pc) {
          constexpr int p = decltype(pc)::value;
          constexpr int n0 = WL ? loads_in_slot(2 * p, DPS, SPAN) : 0;
          constexpr int n1 = WL ? loads_in_slot(2 * p + 1, DPS, SPAN) : 0;
          __builtin_amdgcn_sched_group_barrier(0x008, TN * NPROD, 0);
          if constexpr (n0 > 0) __builtin_amdgcn_sched_group_barrier(0x010, n0, 0);
          if constexpr (p + 1 < NPAIR) __builtin_amdgcn_sched_group_barrier(0x100, PAIR * NAR, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, TN * NPROD, 0);
          if constexpr (n1 > 0) __builtin_amdgcn_sched_group_barrier(0x010, n1, 0);
        });
      };
      pipelined(spread_tag);
    };
    // Stages t whose stage t + NS - 1 exists and is full spread their loads: a prefix, since
    // only the last stage can be partial. Two loops, so that each holds one copy of the body
    // (with both copies in one loop the register allocator spills).
    const int nfull = nst > 0 && !full(nst - 1) ? nst - 1 : nst;
    int t = 0;
    for (; t < nfull - NS + 1; ++t) run_stage(t, std::true_type{});
    for (; t < nst; ++t) run_stage(t, std::false_type{});
  }
}

template <int MODE, typename TC, typename TX, int NS>
__global__ __launch_bounds__(512, 1) void gemm_kernel_dma(GemmBatch batch, const int* done,
                                                          int nsplit, double* ws) {
  if (done && *done) return;
  const GemmOp& op = batch.op[blockIdx.z];
  const int tiles_m = (op.M + DMA_BM - 1) / DMA_BM, tiles_n = (op.N + DMA_BN - 1) / DMA_BN;
  int tm, tn;
  if (!tile_of(tiles_m, tiles_n, tm, tn)) return;
  if (op.tri && tm > tn) return;  // square tiles: wholly below the diagonal, mirrored
  const int ktot = op.K[0] + (op.nseg > 1 ? op.K[1] : 0);
  const int nk = (ktot + DMA_BK - 1) / DMA_BK;
  const int per = (nk + nsplit - 1) / nsplit;
  const int sp = blockIdx.y;
  f4 acc[DMA_TM][DMA_TN];
  gemm_tile_dma_acc<MODE, NS, DmaUser<0, TC, TX>>(op, tm, tn, sp * per * DMA_BK,
                                              min(ktot, (sp + 1) * per * DMA_BK), acc);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  store_acc<MODE, TC, TX, DMA_TM, DMA_TN>(op, acc, tm * DMA_BM + (wave % 2) * DMA_TM * 16,
                                          tn * DMA_BN + (wave / 2) * DMA_TN * 16, lane, sp, nsplit,
                                          ws, blockIdx.z, gridDim.z);
}

// ---- stream-K schedule of the direct-to-LDS tile --------------------------------------------
// T tile-ops (tiles x products, M-fastest within a product) of nk K steps each run on G
// persistent workgroups (G a multiple of 8, one per CU). Rounds r < R = T / G are data
// parallel: workgroup g takes tile-op r G + h(g), where h(g) = (g % 8) (G / 8) + g / 8 keeps 32
// consecutive tile-ops (4 column panels x 8 row tiles sharing operand panels) on one XCD. The
// last T - R G tile-ops (W = (T - R G) nk steps) are cut evenly: workgroup h(g) takes steps
// [h W / G, (h + 1) W / G), at most two tile parts since W / G < nk. A part that is not a whole
// tile leaves its FP32 accumulators in workspace slot 2 h (the first part of h's range) or
// 2 h + 1 (the second); gemm_sk_fixup sums the parts of each cut tile in K order.
constexpr int SK_GRID = 256;  // one workgroup per CU

struct SkArgs {
  int T;       // tile-ops
  int nk;      // K steps per tile
  int R;       // data-parallel rounds
  int64_t W;   // K steps of the cut tile-ops
  int nops;    // products in the launch (tile-ops run through them in order)
};

// Product and tile of tile-op `to` (the products' tile lists concatenated in order).
__device__ __forceinline__ const GemmOp* sk_locate(const GemmBatch& b, int nops, int to, int& tm,
                                                   int& tn) {
  int z = 0;
  for (; z + 1 < nops; ++z) {
    const int c = op_tiles(b.op[z], DMA_BM, DMA_BN);
    if (to < c) break;
    to -= c;
  }
  op_tile(b.op[z], DMA_BM, to, tm, tn);
  return &b.op[z];
}

__device__ __forceinline__ int64_t sk_bound(int64_t W, int h, int G) { return W * h / G; }

template <int MODE, typename TC, typename TX, int NS>
__global__ __launch_bounds__(512, 1) void gemm_kernel_sk(GemmBatch batch, const int* done, SkArgs a,
                                                         float* parts) {
  if (done && *done) return;
  const int G = gridDim.x, g = blockIdx.x;
  const int h = (g & 7) * (G >> 3) + (g >> 3);
  const GemmOp& op0 = batch.op[0];
  const int ktot = op0.K[0] + (op0.nseg > 1 ? op0.K[1] : 0);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  f4 acc[DMA_TM][DMA_TN];
  // One loop over this workgroup's work items (one call site of the tile loop and of the
  // epilogue): first the data-parallel rounds (whole tiles), then its share [u0, u1) of the K
  // steps of the cut tiles.
  const int64_t u0 = sk_bound(a.W, h, G), u1 = sk_bound(a.W, h + 1, G);
  int r = 0, part = 0;
  int64_t u = u0;
  while (r < a.R || u < u1) {
    int to, k0, k1;
    if (r < a.R) {
      to = r * G + h;
      k0 = 0;
      k1 = a.nk;
      ++r;
    } else {
      const int q = (int)(u / a.nk);  // cut tile index
      to = a.R * G + q;
      k0 = (int)(u - (int64_t)q * a.nk);
      k1 = (int)min((int64_t)a.nk, k0 + (u1 - u));
      u += k1 - k0;
    }
    int tm, tn;
    const GemmOp* op = sk_locate(batch, a.nops, to, tm, tn);
    gemm_tile_dma_acc<MODE, NS, DmaUser<1, TC, TX>>(*op, tm, tn, k0 * DMA_BK, min(ktot, k1 * DMA_BK),
                                                acc);
    if (k0 == 0 && k1 == a.nk) {
      store_acc<MODE, TC, TX, DMA_TM, DMA_TN>(*op, acc, tm * DMA_BM + (wave % 2) * DMA_TM * 16,
                                              tn * DMA_BN + (wave / 2) * DMA_TN * 16, lane, 0, 1,
                                              nullptr, 0, 1);
    } else {
      float* slot = parts + (int64_t)(2 * h + part) * (DMA_BM * DMA_BN);
#pragma unroll
      for (int i = 0; i < DMA_TM; ++i)
#pragma unroll
        for (int j = 0; j < DMA_TN; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e)
            slot[((i * DMA_TN + j) * 4 + e) * 512 + threadIdx.x] = acc[i][j][e];
      ++part;
    }
  }
}

// Sums the parts of cut tile blockIdx.x in K order (FP64) and applies the epilogue; blockIdx.y
// takes one of SK_FIX_CHUNKS slices of the tile's elements. Parts and the element each slot
// entry belongs to follow the layout gemm_kernel_sk writes (entry (i TN + j) 4 + r of thread t
// at offset ((i TN + j) 4 + r) 512 + t).
constexpr int SK_FIX_CHUNKS = 32;

template <typename TC, typename TX>
__global__ __launch_bounds__(256) void gemm_sk_fixup(GemmBatch batch, const int* done, SkArgs a,
                                                     int G, const float* parts) {
  if (done && *done) return;
  __shared__ int slot[SK_GRID];
  __shared__ int nslot;
  const int q = blockIdx.x;
  const int64_t s0 = (int64_t)q * a.nk, s1 = s0 + a.nk;
  if (threadIdx.x == 0) {
    // workgroups (in schedule order h) whose share meets [s0, s1), in K order
    int h = (int)((s0 * G) / a.W);
    while (h > 0 && sk_bound(a.W, h, G) > s0) --h;
    while (sk_bound(a.W, h + 1, G) <= s0) ++h;
    int n = 0;
    if (sk_bound(a.W, h + 1, G) < s1) {  // else one workgroup had the whole tile and stored it
      for (; h < G && sk_bound(a.W, h, G) < s1; ++h) {
        const int64_t b = sk_bound(a.W, h, G);
        if (sk_bound(a.W, h + 1, G) <= b) continue;  // empty share
        slot[n++] = 2 * h + (b < s0 ? 1 : 0);
      }
    }
    nslot = n;
  }
  __syncthreads();
  const int n = nslot;
  if (n == 0) return;
  int tm, tn;
  const GemmOp& op = *sk_locate(batch, a.nops, a.R * G + q, tm, tn);
  constexpr int PER = DMA_BM * DMA_BN / SK_FIX_CHUNKS;
  constexpr int U = 4;  // entries per thread and pass, 256 apart (consecutive threads keep
                        // consecutive entries, so loads and stores stay coalesced)
  static_assert(PER % (U * 256) == 0, "whole passes");
  for (int f0 = blockIdx.y * PER + threadIdx.x; f0 < (blockIdx.y + 1) * PER; f0 += U * 256) {
    // the parts are added in K order, U entries at a time (2 U loads in flight)
    double sum[U];
#pragma unroll
    for (int c = 0; c < U; ++c) sum[c] = 0.0;
    int k = 0;
    for (; k + 2 <= n; k += 2) {
      float v[2][U];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int c = 0; c < U; ++c)
          v[u][c] = parts[(int64_t)slot[k + u] * (DMA_BM * DMA_BN) + f0 + 256 * c];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int c = 0; c < U; ++c) sum[c] += (double)v[u][c];
    }
    if (k < n) {
#pragma unroll
      for (int c = 0; c < U; ++c)
        sum[c] += (double)parts[(int64_t)slot[k] * (DMA_BM * DMA_BN) + f0 + 256 * c];
    }
#pragma unroll
    for (int c = 0; c < U; ++c) {
      const int f = f0 + 256 * c;
      const int e = f >> 9, tid = f & 511;  // slot entry and the kernel thread that wrote it
      const int wave = tid >> 6, lane = tid & 63;
      const int i = e / (DMA_TN * 4), j = (e / 4) % DMA_TN, r = e % 4;
      const int row = tm * DMA_BM + (wave % 2) * DMA_TM * 16 + i * 16 + 4 * (lane >> 4) + r;
      const int col = tn * DMA_BN + (wave / 2) * DMA_TN * 16 + j * 16 + (lane & 15);
      if (row < op.M && col < op.N) {
        double v = op.alpha * sum[c];
        if (op.X) v += op.beta * (double)ldg<TX>(op.X, (int64_t)row * op.ldx + col);
        store_out<TC>(op, row, col, v);
      }
    }
  }
}

// Up to 4 same-shape products (blockIdx.z), XCD-remapped tiles (blockIdx.x), split-K (y).
template <int MODE, typename TA, typename TB, typename TC, typename TX, int LA, int LB, int WM,
          int WN, int TM, int TN, int BK, int MINW, bool SWZ = false>
__global__ __launch_bounds__(WM* WN * 64, MINW) void gemm_kernel(GemmBatch batch, const int* done,
                                                                  int nsplit, double* ws) {
  if (done && *done) return;
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16;
  const GemmOp& op = batch.op[blockIdx.z];
  const int tiles_m = (op.M + BM - 1) / BM, tiles_n = (op.N + BN - 1) / BN;
  int tm, tn;
  if (!tile_of(tiles_m, tiles_n, tm, tn)) return;
  // symmetric result: a tile wholly below the diagonal (first row > last column) is mirrored
  if (op.tri && tm * BM > tn * BN + BN - 1) return;
  gemm_tile<MODE, TA, TB, TC, TX, LA, LB, WM, WN, TM, TN, BK, SWZ>(op, tm, tn, blockIdx.y, nsplit,
                                                                  ws, blockIdx.z, gridDim.z);
}

// Tiny products (FP64 and FP32 modes, a few hundred outputs a side, K of a few hundred): one wave
// per 16 x 16 output tile, operands read from memory straight into MFMA fragments (lane l holds
// A(i0 + l % 16, k + l / 16) and B(k + l / 16, j0 + l % 16)), the loads of KU 4-deep K steps
// issued before their MFMAs. A staged macro tile spends such a product waiting on its K loop.
template <int MODE, typename TA, typename TB, typename TC, typename TX, int LA, int LB>
__global__ __launch_bounds__(64) void gemm_kernel_tiny(GemmBatch batch, const int* done,
                                                       int nsplit, double* ws) {
  static_assert(MODE == CF64 || MODE == CF32, "FP64 / FP32 MFMA fragments");
  typedef typename AccT<MODE>::type acc_t;
  typedef typename std::conditional<MODE == CF64, double, float>::type mt;
  if (done && *done) return;
  const GemmOp& op = batch.op[blockIdx.z];
  const int tiles_m = (op.M + 15) / 16, tiles_n = (op.N + 15) / 16;
  int tm, tn;
  if (!tile_of(tiles_m, tiles_n, tm, tn)) return;
  if (op.tri && tm > tn) return;  // written by its mirror tile
  const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
  const int i = tm * 16 + li, j = tn * 16 + li;
  acc_t acc[1][1];
  acc[0][0] = acc_t{0, 0, 0, 0};
  constexpr int KU = 32;
  for (int seg = 0; seg < op.nseg; ++seg) {
    const TA* A = static_cast<const TA*>(op.A[seg]);
    const TB* B = static_cast<const TB*>(op.B[seg]);
    const int64_t lda = op.lda[seg], ldb = op.ldb[seg];
    const int K = op.K[seg];
    for (int k0 = 0; k0 < K; k0 += 4 * KU) {
      mt a[KU], b[KU];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = k0 + 4 * u + lk;
        const bool kin = k < K;
        a[u] = kin && i < op.M
                   ? (mt)(LA == KC ? A[(int64_t)i * lda + k] : A[(int64_t)k * lda + i])
                   : (mt)0;
        b[u] = kin && j < op.N
                   ? (mt)(LB == KC ? B[(int64_t)j * ldb + k] : B[(int64_t)k * ldb + j])
                   : (mt)0;
      }
#pragma unroll
      for (int u = 0; u < KU; ++u) acc[0][0] = mfma4(a[u], b[u], acc[0][0]);
    }
  }
  if (op.tri) {
    // symmetric result: each upper element is also stored to its mirror, in place of the
    // separate mirror pass of the staged tiles
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = MODE == CF64 ? lk + 4 * r : 4 * lk + r;
      const int row = tm * 16 + rr, col = tn * 16 + li;
      if (row < op.M && col < op.N && row <= col) {
        double v = op.alpha * (double)acc[0][0][r];
        if (op.X) v += op.beta * (double)ldg<TX>(op.X, (int64_t)row * op.ldx + col);
        store_out<TC>(op, row, col, v);
        if (row < col) store_out<TC>(op, col, row, v);
      }
    }
    return;
  }
  store_acc<MODE, TC, TX, 1, 1>(op, acc, tm * 16, tn * 16, lane, 0, 1, ws, blockIdx.z,
                                gridDim.z);
}

// Grouped products of uneven shapes: a persistent grid walks the concatenated tile list of all
// ops (tile_start = prefix sums); an op whose `done` flag is set is skipped.
struct GroupedArgs {
  const GemmOp* ops;
  const int* tile_start;  // nops + 1 entries
  const int* const* done; // per op, nullable entries
  int nops;
};

template <int MODE, typename TA, typename TB, typename TC, typename TX, int LA, int LB, int WM,
          int WN, int TM, int TN, int BK, int MINW, bool SWZ = false>
__global__ __launch_bounds__(WM* WN * 64, MINW) void gemm_grouped_kernel(GroupedArgs g) {
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16;
  const int total = g.tile_start[g.nops];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int lo = 0, hi = g.nops - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (g.tile_start[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int* dn = g.done[lo];
    if (dn && *dn) continue;
    const GemmOp& op = g.ops[lo];  // by reference: a local copy would sit in scratch memory
    const int tiles_m = (op.M + BM - 1) / BM;
    const int local = t - g.tile_start[lo];
    gemm_tile<MODE, TA, TB, TC, TX, LA, LB, WM, WN, TM, TN, BK, SWZ>(
        op, local % tiles_m, local / tiles_m, 0, 1, nullptr, 0, 1);
    __syncthreads();  // LDS is reused by the next tile
  }
}

typedef void (*grouped_fn)(GroupedArgs);
typedef void (*sk_fn)(GemmBatch, const int*, SkArgs, float*);
typedef void (*sk_fixup_fn)(GemmBatch, const int*, SkArgs, int, const float*);

template <int MODE, typename TC, typename TX>
sk_fn pick_sk_kernel() {
  return gemm_kernel_sk<MODE, TC, TX, dma_stages(MODE)>;
}

// Tile shapes (macro tile M x N): 0: 128x128 (4 waves), 1: 64x64 (4 waves, 2 workgroups per
// CU), 2: 256x128 (8 waves), 3: 128x256 (8 waves), 4: BF16x3: 256x256 (8 waves of 128x64,
// swizzled unpadded LDS); FP64/FP32: 128x128 with 2 workgroups per CU. 5: BF16 modes on planes
// with both operands k-contiguous: the 256x256 tile fed by direct-to-LDS loads (3 stages for the
// two-product modes, 2 for BF16x3).
//    6: tile 5 on a stream-K schedule (persistent, whole-tile rounds, then the remaining tiles
//       cut evenly across the workgroups).
//    7: FP64 / FP32 only: 16 x 16, one wave per tile, fragments loaded from memory
//       (gemm_kernel_tiny), no split-K.
constexpr int NTILES = 8;
constexpr int NTILES_GROUPED = 5;
inline bool tile_big(int t, int mode) { return t >= 4 && is_bf16_mode(mode); }
inline int tile_bm(int t, int mode) {
  return t == 7 ? 16 : t == 1 ? 64 : (t == 2 || tile_big(t, mode) ? 256 : 128);
}
inline int tile_bn(int t, int mode) {
  return t == 7 ? 16 : t == 1 ? 64 : (t == 3 || tile_big(t, mode) ? 256 : 128);
}
inline int tile_threads(int t, int mode) {
  return t == 7 ? 64 : (t == 2 || t == 3 || tile_big(t, mode)) ? 512 : 256;
}

template <int MODE, typename TA, typename TB, typename TC, typename TX, int LA, int LB>
grouped_fn pick_grouped_tile(int tile) {
  constexpr int BK = is_bf16_mode(MODE) ? 32 : 16;
  switch (tile) {
    case 0: return gemm_grouped_kernel<MODE, TA, TB, TC, TX, LA, LB, 2, 2, 4, 4, BK, 1>;
    case 1: return gemm_grouped_kernel<MODE, TA, TB, TC, TX, LA, LB, 2, 2, 2, 2, BK, 2>;
    case 2: return gemm_grouped_kernel<MODE, TA, TB, TC, TX, LA, LB, 4, 2, 4, 4, BK, 1>;
    case 3: return gemm_grouped_kernel<MODE, TA, TB, TC, TX, LA, LB, 2, 4, 4, 4, BK, 1>;
    case 4:
      if constexpr (is_bf16_mode(MODE))
        return gemm_grouped_kernel<MODE, TA, TB, TC, TX, LA, LB, 2, 4, 8, 4, BK, 1, true>;
      else
        return gemm_grouped_kernel<MODE, TA, TB, TC, TX, LA, LB, 2, 2, 4, 4, BK, 2>;
    default: return nullptr;
  }
}

template <int MODE, typename TA, typename TB, typename TC, typename TX, int LA, int LB>
gemm_fn pick_tile(int tile) {
  constexpr int BK = is_bf16_mode(MODE) ? 32 : 16;
  switch (tile) {
    case 0: return gemm_kernel<MODE, TA, TB, TC, TX, LA, LB, 2, 2, 4, 4, BK, 1>;
    case 1: return gemm_kernel<MODE, TA, TB, TC, TX, LA, LB, 2, 2, 2, 2, BK, 2>;
    case 2: return gemm_kernel<MODE, TA, TB, TC, TX, LA, LB, 4, 2, 4, 4, BK, 1>;
    case 3: return gemm_kernel<MODE, TA, TB, TC, TX, LA, LB, 2, 4, 4, 4, BK, 1>;
    case 4:
      if constexpr (is_bf16_mode(MODE))
        return gemm_kernel<MODE, TA, TB, TC, TX, LA, LB, 2, 4, 8, 4, BK, 1, true>;
      else
        return gemm_kernel<MODE, TA, TB, TC, TX, LA, LB, 2, 2, 4, 4, BK, 2>;
    case 5:
      if constexpr (is_bf16_mode(MODE) && std::is_same<TA, unsigned short>::value &&
                    std::is_same<TB, unsigned short>::value && LA == KC && LB == KC)
        return gemm_kernel_dma<MODE, TC, TX, dma_stages(MODE)>;
      else
        return nullptr;
    case 7:
      if constexpr (MODE == CF64 || MODE == CF32)
        return gemm_kernel_tiny<MODE, TA, TB, TC, TX, LA, LB>;
      else
        return nullptr;
    default: return nullptr;
  }
}

template <int MODE, typename TA, typename TB, typename TC, typename TX>
gemm_fn pick_layout(int la, int lb, int tile) {
  if (la == KC && lb == KC) return pick_tile<MODE, TA, TB, TC, TX, KC, KC>(tile);
  if (la == KC && lb == RC) return pick_tile<MODE, TA, TB, TC, TX, KC, RC>(tile);
  if (la == RC && lb == RC) return pick_tile<MODE, TA, TB, TC, TX, RC, RC>(tile);
  return nullptr;
}

}  // namespace gemm_detail
}  // namespace omm
