// MFMA GEMMs for gfx950: C = alpha * sum_seg A_seg * B_seg + beta * X.
//
// Every cubic-scaling product of the method goes through here: the operator products
// C*[Hs|S], D*[Hs|S] and G*P (M x N x N), the projections D*[HC;SC;HD;SD]^T (M x M x N), the
// gradient HW*SC + SW*HC (M x N x M) and the rank-nb updates of the preconditioner inversion.
//
// Three compute modes share one tile loop:
//   CF64    v_mfma_f64_16x16x4f64, FP64 operands and accumulators;
//   CF32    v_mfma_f32_16x16x4f32, operands rounded to FP32, FP32 accumulators;
//   CBF16X3 v_mfma_f32_16x16x32_bf16 on a hi/lo split of each FP32 operand
//           (a = a_hi + a_lo with a_hi = bf16(a), a_lo = bf16(a - a_hi)), three products
//           a_hi b_hi + a_hi b_lo + a_lo b_hi per K step, FP32 accumulators. The split is done
//           while staging a tile into LDS, so operands stay FP32 (or FP64) in HBM.
//
// Workgroups are 256 threads (2 x 2 waves). Macro tiles are 128 x 128 (each wave 64 x 64, i.e.
// 4 x 4 MFMA blocks) or 64 x 64. Operand tiles are staged through LDS with one tile of register
// prefetch. The linear workgroup id is remapped so that each of the 8 XCDs receives a contiguous
// run of tiles ordered down the M dimension: tiles that share a column panel of the (large) B
// operand run on the same XCD at the same time and share its L2.
#include "omm_internal.h"

namespace omm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

struct GemmBatch {
  GemmOp op[4];
};

template <typename T>
struct AccOf;
template <>
struct AccOf<double> {
  typedef d4 type;
};
template <>
struct AccOf<float> {
  typedef f4 type;
};

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ T ld(const void* p, int64_t i) {
  return static_cast<const T*>(p)[i];
}

// bf16 bits of a float, round to nearest even (finite inputs).
__device__ __forceinline__ unsigned short bf16_bits(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_float(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}

// Map the linear workgroup id to a (tm, tn) tile, contiguous per XCD, M fastest.
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

// K range [kb, ke) of segment `seg` owned by split `sp` of `nsplit` (splits cut the concatenated
// K of all segments into BK-aligned chunks).
template <int BK>
__device__ __forceinline__ void split_range(const GemmOp& op, int seg, int sp, int nsplit, int& kb,
                                            int& ke) {
  const int ktot = op.K[0] + (op.nseg > 1 ? op.K[1] : 0);
  const int nk = (ktot + BK - 1) / BK;
  const int per = (nk + nsplit - 1) / nsplit;
  int g0 = sp * per * BK, g1 = min(ktot, (sp + 1) * per * BK);
  const int off = seg == 0 ? 0 : op.K[0];
  kb = max(g0 - off, 0);
  ke = min(g1 - off, op.K[seg]);
}

// ----------------------------------------------------------------------------------------------
// FP64 / FP32 MFMA (16x16x4) tile loop.
template <typename CT, typename TA, typename TB, typename TC, typename TX, int LA, int LB, int TMN>
__global__ __launch_bounds__(256) void gemm_k4(GemmBatch batch, const int* done, int nsplit,
                                               double* ws) {
  if (done && *done) return;
  constexpr int TM = TMN, TN = TMN;  // MFMA blocks per wave
  constexpr int BM = 2 * TM * 16, BN = 2 * TN * 16, BK = 16, PAD = 16;
  constexpr int LA_PER = BM * BK / 256, LB_PER = BN * BK / 256;
  typedef typename AccOf<CT>::type acc_t;

  const GemmOp& op = batch.op[blockIdx.z];
  const int tiles_m = (op.M + BM - 1) / BM, tiles_n = (op.N + BN - 1) / BN;
  int tm, tn;
  if (!tile_of(tiles_m, tiles_n, tm, tn)) return;
  const int sp = blockIdx.y;
  const int m0 = tm * BM, n0 = tn * BN;

  __shared__ CT As[BK][BM + PAD];
  __shared__ CT Bs[BK][BN + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  acc_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  for (int seg = 0; seg < op.nseg; ++seg) {
    int kb, ke;
    split_range<BK>(op, seg, sp, nsplit, kb, ke);
    if (kb >= ke) continue;
    const void* A = op.A[seg];
    const void* B = op.B[seg];
    const int64_t lda = op.lda[seg], ldb = op.ldb[seg];
    CT ra[LA_PER], rb[LB_PER];
    auto load = [&](int k0) {
#pragma unroll
      for (int i = 0; i < LA_PER; ++i) {
        const int e = tid + i * 256;
        int r, k;
        if (LA == KC) { r = e / BK; k = e % BK; } else { r = e % BM; k = e / BM; }
        const int gr = m0 + r, gk = k0 + k;
        CT v = 0;
        if (gr < op.M && gk < ke)
          v = (CT)ld<TA>(A, LA == KC ? (int64_t)gr * lda + gk : (int64_t)gk * lda + gr);
        ra[i] = v;
      }
#pragma unroll
      for (int i = 0; i < LB_PER; ++i) {
        const int e = tid + i * 256;
        int r, k;
        if (LB == KC) { r = e / BK; k = e % BK; } else { r = e % BN; k = e / BN; }
        const int gr = n0 + r, gk = k0 + k;
        CT v = 0;
        if (gr < op.N && gk < ke)
          v = (CT)ld<TB>(B, LB == KC ? (int64_t)gr * ldb + gk : (int64_t)gk * ldb + gr);
        rb[i] = v;
      }
    };
    load(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
      __syncthreads();
#pragma unroll
      for (int i = 0; i < LA_PER; ++i) {
        const int e = tid + i * 256;
        if (LA == KC) As[e % BK][e / BK] = ra[i]; else As[e / BM][e % BM] = ra[i];
      }
#pragma unroll
      for (int i = 0; i < LB_PER; ++i) {
        const int e = tid + i * 256;
        if (LB == KC) Bs[e % BK][e / BK] = rb[i]; else Bs[e / BN][e % BN] = rb[i];
      }
      __syncthreads();
      if (k0 + BK < ke) load(k0 + BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        CT a[TM], b[TN];
        const int kr = kk + (lane >> 4);
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = As[kr][wm * TM * 16 + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = Bs[kr][wn * TN * 16 + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
      }
    }
  }

  // Epilogue: lane holds column lane%16 of each 16x16 block; its 4 accumulator values are rows
  // 4*(lane/16)+r for the FP32 instruction and rows lane/16+4r for the FP64 one.
  const int nops = gridDim.z;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = sizeof(CT) == 8 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
        const int row = m0 + wm * TM * 16 + i * 16 + rr;
        const int col = n0 + wn * TN * 16 + j * 16 + (lane & 15);
        if (row < op.M && col < op.N) {
          const double s = (double)acc[i][j][r];
          if (nsplit > 1) {
            ws[((int64_t)sp * nops + blockIdx.z) * op.M * op.N + (int64_t)row * op.N + col] = s;
          } else {
            double v = op.alpha * s;
            if (op.X) v += op.beta * (double)ld<TX>(op.X, (int64_t)row * op.ldx + col);
            static_cast<TC*>(op.C)[(int64_t)row * op.ldc + col] = (TC)v;
          }
        }
      }
}

// ----------------------------------------------------------------------------------------------
// BF16x3 split MFMA (16x16x32) tile loop. LDS holds hi and lo parts, k contiguous per row so a
// lane's 8 consecutive k values are one 16-byte read.
template <typename TA, typename TB, typename TC, typename TX, int LA, int LB, int TMN>
__global__ __launch_bounds__(256) void gemm_bf16x3(GemmBatch batch, const int* done, int nsplit,
                                                   double* ws) {
  if (done && *done) return;
  constexpr int TM = TMN, TN = TMN;
  constexpr int BM = 2 * TM * 16, BN = 2 * TN * 16, BK = 32, RS = BK + 8;  // RS: row stride
  constexpr int LA_PER = BM * BK / 256, LB_PER = BN * BK / 256;

  const GemmOp& op = batch.op[blockIdx.z];
  const int tiles_m = (op.M + BM - 1) / BM, tiles_n = (op.N + BN - 1) / BN;
  int tm, tn;
  if (!tile_of(tiles_m, tiles_n, tm, tn)) return;
  const int sp = blockIdx.y;
  const int m0 = tm * BM, n0 = tn * BN;

  __shared__ __attribute__((aligned(16))) unsigned short Ah[BM * RS], Al[BM * RS];
  __shared__ __attribute__((aligned(16))) unsigned short Bh[BN * RS], Bl[BN * RS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0, 0, 0, 0};

  for (int seg = 0; seg < op.nseg; ++seg) {
    int kb, ke;
    split_range<BK>(op, seg, sp, nsplit, kb, ke);
    if (kb >= ke) continue;
    const void* A = op.A[seg];
    const void* B = op.B[seg];
    const int64_t lda = op.lda[seg], ldb = op.ldb[seg];
    float ra[LA_PER], rb[LB_PER];
    auto load = [&](int k0) {
#pragma unroll
      for (int i = 0; i < LA_PER; ++i) {
        const int e = tid + i * 256;
        int r, k;
        if (LA == KC) { r = e / BK; k = e % BK; } else { r = e % BM; k = e / BM; }
        const int gr = m0 + r, gk = k0 + k;
        float v = 0.f;
        if (gr < op.M && gk < ke)
          v = (float)ld<TA>(A, LA == KC ? (int64_t)gr * lda + gk : (int64_t)gk * lda + gr);
        ra[i] = v;
      }
#pragma unroll
      for (int i = 0; i < LB_PER; ++i) {
        const int e = tid + i * 256;
        int r, k;
        if (LB == KC) { r = e / BK; k = e % BK; } else { r = e % BN; k = e / BN; }
        const int gr = n0 + r, gk = k0 + k;
        float v = 0.f;
        if (gr < op.N && gk < ke)
          v = (float)ld<TB>(B, LB == KC ? (int64_t)gr * ldb + gk : (int64_t)gk * ldb + gr);
        rb[i] = v;
      }
    };
    load(kb);
    for (int k0 = kb; k0 < ke; k0 += BK) {
      __syncthreads();
#pragma unroll
      for (int i = 0; i < LA_PER; ++i) {
        const int e = tid + i * 256;
        int r, k;
        if (LA == KC) { r = e / BK; k = e % BK; } else { r = e % BM; k = e / BM; }
        const unsigned short h = bf16_bits(ra[i]);
        Ah[r * RS + k] = h;
        Al[r * RS + k] = bf16_bits(ra[i] - bf16_to_float(h));
      }
#pragma unroll
      for (int i = 0; i < LB_PER; ++i) {
        const int e = tid + i * 256;
        int r, k;
        if (LB == KC) { r = e / BK; k = e % BK; } else { r = e % BN; k = e / BN; }
        const unsigned short h = bf16_bits(rb[i]);
        Bh[r * RS + k] = h;
        Bl[r * RS + k] = bf16_bits(rb[i] - bf16_to_float(h));
      }
      __syncthreads();
      if (k0 + BK < ke) load(k0 + BK);
      const int kof = 8 * (lane >> 4);
      bf8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int r = wm * TM * 16 + i * 16 + (lane & 15);
        ah[i] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&Ah[r * RS + kof]));
        al[i] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&Al[r * RS + kof]));
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int r = wn * TN * 16 + j * 16 + (lane & 15);
        bh[j] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&Bh[r * RS + kof]));
        bl[j] = __builtin_bit_cast(bf8, *reinterpret_cast<const u16x8*>(&Bl[r * RS + kof]));
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
  }

  const int nops = gridDim.z;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * TM * 16 + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn * TN * 16 + j * 16 + (lane & 15);
        if (row < op.M && col < op.N) {
          const double s = (double)acc[i][j][r];
          if (nsplit > 1) {
            ws[((int64_t)sp * nops + blockIdx.z) * op.M * op.N + (int64_t)row * op.N + col] = s;
          } else {
            double v = op.alpha * s;
            if (op.X) v += op.beta * (double)ld<TX>(op.X, (int64_t)row * op.ldx + col);
            static_cast<TC*>(op.C)[(int64_t)row * op.ldc + col] = (TC)v;
          }
        }
      }
}

// Sum split-K partials in split order (deterministic) and apply the epilogue.
template <typename TC, typename TX>
__global__ __launch_bounds__(256) void splitk_reduce(GemmBatch batch, const int* done, int nsplit,
                                                     const double* ws) {
  if (done && *done) return;
  const GemmOp& op = batch.op[blockIdx.y];
  const int64_t mn = (int64_t)op.M * op.N;
  const int nops = gridDim.y;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < mn;
       idx += (int64_t)gridDim.x * 256) {
    double s = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) s += ws[((int64_t)sp * nops + blockIdx.y) * mn + idx];
    const int row = (int)(idx / op.N), col = (int)(idx % op.N);
    double v = op.alpha * s;
    if (op.X) v += op.beta * (double)ld<TX>(op.X, (int64_t)row * op.ldx + col);
    static_cast<TC*>(op.C)[(int64_t)row * op.ldc + col] = (TC)v;
  }
}

template <typename T>
struct TypeOf;

typedef void (*gemm_fn)(GemmBatch, const int*, int, double*);

template <int C, typename TA, typename TB, typename TC, typename TX, int LA, int LB, int TMN>
gemm_fn pick_kernel() {
  if constexpr (C == CF64) {
    return gemm_k4<double, TA, TB, TC, TX, LA, LB, TMN>;
  } else if constexpr (C == CF32) {
    return gemm_k4<float, TA, TB, TC, TX, LA, LB, TMN>;
  } else {
    return gemm_bf16x3<TA, TB, TC, TX, LA, LB, TMN>;
  }
}

template <int C, typename TA, typename TB, typename TC, typename TX>
gemm_fn pick_layout(int la, int lb, int tile) {
#define OMM_PICK(LA_, LB_)                                                      \
  if (la == LA_ && lb == LB_) {                                                 \
    return tile == 1 ? pick_kernel<C, TA, TB, TC, TX, LA_, LB_, 2>()            \
                     : pick_kernel<C, TA, TB, TC, TX, LA_, LB_, 4>();           \
  }
  OMM_PICK(KC, KC)
  OMM_PICK(KC, RC)
  OMM_PICK(RC, KC)
  OMM_PICK(RC, RC)
#undef OMM_PICK
  return nullptr;
}

template <int C>
gemm_fn pick_types(const GemmDesc& d) {
  if constexpr (C == CF64) {
    if (d.ta == T_F64 && d.tb == T_F64 && d.tc == T_F64 && d.tx == T_F64)
      return pick_layout<C, double, double, double, double>(d.la, d.lb, d.tile);
    return nullptr;
  } else {
    if (d.ta == T_F32 && d.tb == T_F32 && d.tc == T_F32 && d.tx == T_F32)
      return pick_layout<C, float, float, float, float>(d.la, d.lb, d.tile);
    if (d.ta == T_F32 && d.tb == T_F32 && d.tc == T_F64 && d.tx == T_F64)
      return pick_layout<C, float, float, double, double>(d.la, d.lb, d.tile);
    if (d.ta == T_F64 && d.tb == T_F32 && d.tc == T_F32 && d.tx == T_F32)
      return pick_layout<C, double, float, float, float>(d.la, d.lb, d.tile);
    return nullptr;
  }
}

}  // namespace

size_t gemm_splitk_ws_bytes(const GemmOp* ops, int nops, int splitk) {
  if (splitk <= 1) return 0;
  return (size_t)splitk * nops * (size_t)ops[0].M * ops[0].N * sizeof(double);
}

hipError_t gemm_launch(const GemmDesc& d, const GemmOp* ops, int nops, const int* done, double* ws,
                       size_t ws_bytes, hipStream_t s) {
  if (nops < 1 || nops > 4) return hipErrorInvalidValue;
  GemmBatch b;
  for (int i = 0; i < nops; ++i) {
    b.op[i] = ops[i];
    if (ops[i].M != ops[0].M || ops[i].N != ops[0].N) return hipErrorInvalidValue;
    if (ops[i].nseg < 1 || ops[i].nseg > 2) return hipErrorInvalidValue;
  }
  const int M = ops[0].M, N = ops[0].N;
  if (M <= 0 || N <= 0) return hipSuccess;
  gemm_fn fn = nullptr;
  if (d.compute == CF64) fn = pick_types<CF64>(d);
  else if (d.compute == CF32) fn = pick_types<CF32>(d);
  else if (d.compute == CBF16X3) fn = pick_types<CBF16X3>(d);
  if (!fn) return hipErrorInvalidValue;
  const int bm = d.tile == 1 ? 64 : 128;
  const int tiles = ((M + bm - 1) / bm) * ((N + bm - 1) / bm);
  const int per = (tiles + 7) / 8;
  int splitk = d.splitk > 1 ? d.splitk : 1;
  if (splitk > 1) {
    if (!ws || ws_bytes < gemm_splitk_ws_bytes(ops, nops, splitk)) return hipErrorInvalidValue;
  }
  dim3 grid(8 * per, splitk, nops);
  hipLaunchKernelGGL(fn, grid, dim3(256), 0, s, b, done, splitk, ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splitk == 1) return e;
  const int64_t mn = (int64_t)M * N;
  int blocks = (int)((mn + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  dim3 rgrid(blocks, nops);
  void (*red)(GemmBatch, const int*, int, const double*) = nullptr;
  if (d.tc == T_F64) red = d.tx == T_F64 ? splitk_reduce<double, double> : splitk_reduce<double, float>;
  else red = d.tx == T_F64 ? splitk_reduce<float, double> : splitk_reduce<float, float>;
  hipLaunchKernelGGL(red, rgrid, dim3(256), 0, s, b, done, splitk, (const double*)ws);
  return hipGetLastError();
}

}  // namespace omm
