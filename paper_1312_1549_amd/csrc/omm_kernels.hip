// Memory-bound stages of one CG line search (Sec. 2.3 of the paper): FP64 reductions for the
// Polak-Ribiere coefficient and the quartic coefficients (Eq. 13), the device-side line
// minimum, and the updates of Eq. 16. All reductions are two-pass with a fixed grid, so a rerun
// is bitwise identical. The scalar state of a minimization lives in device memory (DevState);
// no stage needs the host.
#include <math.h>

#include <algorithm>

#include "omm_internal.h"

namespace omm {
namespace {

constexpr int NT = 256;
// block-reduction scratch: up to NCOEF values at once (block_sums), one slot per wave each
constexpr int SH_SUMS = NCOEF * (NT / 64);

// Sum of `v` over the block (FP64, fixed order). Result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) t += sh[i];
  return t;
}

// block_sum of W values at once (each in block_sum's order: the same results), with one pair of
// barriers instead of W; sh holds W * NT / 64 doubles. Results valid in thread 0.
template <int W>
__device__ __forceinline__ void block_sums(double (&v)[W], double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int k = 0; k < W; ++k) v[k] += __shfl_down(v[k], o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < W; ++k) sh[k * (NT / 64) + w] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < W; ++k) {
      double t = 0.0;
      for (int i = 0; i < NT / 64; ++i) t += sh[k * (NT / 64) + i];
      v[k] = t;
    }
}

// Fixed-order sum over nb partial rows (stride w) of column c, by the whole block; result in
// thread 0. Each thread sums a strided subset in index order, then block_sum combines them.
__device__ __forceinline__ double sum_partials(const double* partials, int nb, int w, int c,
                                               double* sh) {
  double v = 0.0;
  for (int b = threadIdx.x; b < nb; b += NT) v += partials[b * w + c];
  return block_sum(v, sh);
}

// sum_partials of columns 0..W-1 of rows of width W, in the same per-column order, with the
// loads of all columns in flight together.
template <int W>
__device__ __forceinline__ void sum_partials_all(const double* partials, int nb, double* sh,
                                                 double (&out)[W]) {
  double v[W];
#pragma unroll
  for (int k = 0; k < W; ++k) v[k] = 0.0;
  for (int b = threadIdx.x; b < nb; b += NT)
#pragma unroll
    for (int k = 0; k < W; ++k) v[k] += partials[b * W + k];
  block_sums<W>(v, sh);
#pragma unroll
  for (int k = 0; k < W; ++k) out[k] = v[k];
}

int red_blocks(int64_t n) {
  int64_t b = (n + NT - 1) / NT;
  if (b > RED_BLOCKS) b = RED_BLOCKS;
  if (b < 1) b = 1;
  return (int)b;
}

__global__ void k_shift(const double* H, const double* S, double eta, double* Hs, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    Hs[i] = H[i] - eta * S[i];
}

template <typename A, typename B>
__global__ void k_convert(const A* src, B* dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    dst[i] = (B)src[i];
}

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// hi/lo bf16 planes of src (rows x cols, contiguous) into rows of length ld >= cols (ld a
// multiple of 4): rows blockIdx.y, blockIdx.y + gridDim.y, .., 4 elements per thread (8-byte
// stores).
template <typename T>
__global__ void k_split(const T* src, unsigned short* hi, unsigned short* lo, int64_t rows,
                        int64_t cols, int64_t ld, const DevState* st) {
  if (st && st->done) return;
  typedef unsigned short us4 __attribute__((ext_vector_type(4)));
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
    const T* srow = src + r * cols;
    for (int64_t c4 = ((int64_t)blockIdx.x * NT + threadIdx.x) * 4; c4 < cols;
         c4 += (int64_t)gridDim.x * NT * 4) {
      if (c4 + 4 <= cols) {
        us4 h, l;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double v = (double)srow[c4 + u];
          const unsigned short hb = bf16_bits((float)v);
          h[u] = hb;
          l[u] = bf16_bits((float)(v - (double)__uint_as_float(((unsigned int)hb) << 16)));
        }
        *reinterpret_cast<us4*>(hi + r * ld + c4) = h;
        *reinterpret_cast<us4*>(lo + r * ld + c4) = l;
      } else {
        for (int64_t c = c4; c < cols; ++c) {
          const double v = (double)srow[c];
          const unsigned short hb = bf16_bits((float)v);
          hi[r * ld + c] = hb;
          lo[r * ld + c] = bf16_bits((float)(v - (double)__uint_as_float(((unsigned int)hb) << 16)));
        }
      }
    }
  }
}

// Transposing split through a 32 x 33 LDS tile: dst (cols x rows, row length ld) = planes of
// src^T.
template <typename T>
__global__ void k_split_t(const T* src, unsigned short* hi, unsigned short* lo, int rows, int cols,
                          int64_t ld, const DevState* st) {
  if (st && st->done) return;
  __shared__ T t[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int gr = r0 + r, gc = c0 + tx;
    t[r][tx] = (gr < rows && gc < cols) ? src[(int64_t)gr * cols + gc] : (T)0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int oc = c0 + r, orow = r0 + tx;  // output row oc (a source column), column orow
    if (oc < cols && orow < rows) {
      const double v = (double)t[tx][r];
      const unsigned short hb = bf16_bits((float)v);
      const int64_t o = (int64_t)oc * ld + orow;
      hi[o] = hb;
      lo[o] = bf16_bits((float)(v - (double)__uint_as_float(((unsigned int)hb) << 16)));
    }
  }
}

int ew_blocks(int64_t n) {
  int64_t b = (n + NT - 1) / NT;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

// flags[0] |= non-finite entry, flags[1] |= |a_ij - a_ji| > rtol * max(1, |a_ij|, |a_ji|).
__global__ void k_validate(const double* A, int64_t n, double rtol, int* flags) {
  __shared__ double t[32][33];
  const int64_t bi = (int64_t)blockIdx.y * 32, bj = (int64_t)blockIdx.x * 32;
  if (bj < bi) return;  // upper block triangle (incl. diagonal blocks) covers every pair
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bj + r, j = bi + tx;  // transposed tile (bj, bi)
    t[r][tx] = (i < n && j < n) ? A[i * n + j] : 0.0;
  }
  __syncthreads();
  int bad_f = 0, bad_s = 0;
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bi + r, j = bj + tx;
    if (i < n && j < n) {
      const double a = A[i * n + j], b = t[tx][r];
      if (!isfinite(a)) bad_f = 1;
      const double m = fmax(1.0, fmax(fabs(a), fabs(b)));
      if (!(fabs(a - b) <= rtol * m)) bad_s = 1;
    }
  }
  if (bad_f) atomicOr(&flags[0], 1);
  if (bad_s) atomicOr(&flags[1], 1);
}

// A <- (A + A^T) / 2; one thread per unordered pair.
__global__ void k_symmetrize(double* A, int64_t n) {
  __shared__ double t[32][33];
  const int64_t bi = (int64_t)blockIdx.y * 32, bj = (int64_t)blockIdx.x * 32;
  if (bj < bi) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // load transposed tile (bj, bi) and this tile (bi, bj); write both halves
  __shared__ double u[32][33];
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bj + r, j = bi + tx;
    t[r][tx] = (i < n && j < n) ? A[i * n + j] : 0.0;
    const int64_t i2 = bi + r, j2 = bj + tx;
    u[r][tx] = (i2 < n && j2 < n) ? A[i2 * n + j2] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bi + r, j = bj + tx;
    if (i < n && j < n) {
      if (bi == bj && j < i) continue;  // diagonal block: each pair once (j >= i)
      const double v = 0.5 * (u[r][tx] + t[tx][r]);
      A[i * n + j] = v;
      A[j * n + i] = v;
    }
  }
}

// ---- energy of (HW, SW): Eq. 8 -----------------------------------------------------------------
__device__ __forceinline__ void b_energy_partials(const double* HW, const double* SW, int M, double* partials, int bid, int nb) {
  __shared__ double sh[SH_SUMS];
  const int64_t n = (int64_t)M * M;
  double tr = 0.0, f = 0.0, trs = 0.0;
  for (int64_t i = (int64_t)bid * NT + threadIdx.x; i < n; i += (int64_t)nb * NT) {
    const int r = (int)(i / M), c = (int)(i % M);
    const double h = HW[i], s = SW[i];
    f += s * h;
    if (r == c) { tr += h; trs += s; }
  }
  double v3[3] = {tr, f, trs};
  block_sums<3>(v3, sh);
  const double a = v3[0], b = v3[1], c = v3[2];
  if (threadIdx.x == 0) {
    partials[bid * 3 + 0] = a;
    partials[bid * 3 + 1] = b;
    partials[bid * 3 + 2] = c;
  }
}

__global__ void k_energy_partials(const double* HW, const double* SW, int M, double* partials) {
  b_energy_partials(HW, SW, M, partials, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ void f_energy_init_final(const double* partials, int nb, DevState* st, double* trace) {
  __shared__ double sh[SH_SUMS];
  const double tr = sum_partials(partials, nb, 3, 0, sh);
  const double f = sum_partials(partials, nb, 3, 1, sh);
  if (threadIdx.x != 0) return;
  const double E = 4.0 * tr - 2.0 * f;
  st->E = E;
  st->E_prev = E;
  if (trace) trace[0] = E;
  if (!isfinite(E)) st->done = -5;
}

__global__ void k_energy_init_final(const double* partials, int nb, DevState* st, double* trace) {
  f_energy_init_final(partials, nb, st, trace);
}

// ---- Polak-Ribiere coefficient and direction ----------------------------------------------------
template <typename T, typename TP = T>
__device__ __forceinline__ void b_pr_partials(const T* G, const TP* PG, const T* Gp, int64_t n, int first,
                              double* partials, const DevState* st, int bid, int nb) {
  if (st->done) return;
  __shared__ double sh[SH_SUMS];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)bid * NT + threadIdx.x; i < n; i += (int64_t)nb * NT) {
    const double pg = (double)PG[i];
    s1 += pg * (double)G[i];
    if (!first) s2 += pg * (double)Gp[i];
  }
  double v2[2] = {s1, s2};
  block_sums<2>(v2, sh);
  const double a = v2[0], b = v2[1];
  if (threadIdx.x == 0) {
    partials[bid * 2 + 0] = a;
    partials[bid * 2 + 1] = b;
  }
}

template <typename T, typename TP>
__global__ void k_pr_partials(const T* G, const TP* PG, const T* Gp, int64_t n, int first,
                              double* partials, const DevState* st) {
  b_pr_partials(G, PG, Gp, n, first, partials, st, blockIdx.x, gridDim.x);
}

// The same sums four elements per load (arrays 4-element aligned; the tail past the last full
// group of four is added by block 0), two groups in flight per thread.
template <typename TG, typename TP>
__global__ void k_pr_partials4(const TG* G, const TP* PG, const TG* Gp, int64_t n, int first,
                               double* partials, const DevState* st) {
  if (st->done) return;
  typedef TG G4 __attribute__((ext_vector_type(4)));
  typedef TP P4 __attribute__((ext_vector_type(4)));
  __shared__ double sh[SH_SUMS];
  const int64_t n4 = n / 4, stride = (int64_t)gridDim.x * NT;
  const G4* g4 = reinterpret_cast<const G4*>(G);
  const G4* q4 = reinterpret_cast<const G4*>(Gp);
  const P4* p4 = reinterpret_cast<const P4*>(PG);
  double s1 = 0.0, s2 = 0.0;
  int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  for (; i + stride < n4; i += 2 * stride) {
    const P4 pa = p4[i], pb = p4[i + stride];
    const G4 ga = g4[i], gb = g4[i + stride];
    s1 += (double)pa.x * ga.x + (double)pa.y * ga.y + (double)pa.z * ga.z + (double)pa.w * ga.w;
    s1 += (double)pb.x * gb.x + (double)pb.y * gb.y + (double)pb.z * gb.z + (double)pb.w * gb.w;
    if (!first) {
      const G4 qa = q4[i], qb = q4[i + stride];
      s2 += (double)pa.x * qa.x + (double)pa.y * qa.y + (double)pa.z * qa.z + (double)pa.w * qa.w;
      s2 += (double)pb.x * qb.x + (double)pb.y * qb.y + (double)pb.z * qb.z + (double)pb.w * qb.w;
    }
  }
  if (i < n4) {
    const P4 pa = p4[i];
    const G4 ga = g4[i];
    s1 += (double)pa.x * ga.x + (double)pa.y * ga.y + (double)pa.z * ga.z + (double)pa.w * ga.w;
    if (!first) {
      const G4 qa = q4[i];
      s2 += (double)pa.x * qa.x + (double)pa.y * qa.y + (double)pa.z * qa.z + (double)pa.w * qa.w;
    }
  }
  if (blockIdx.x == 0)
    for (int64_t j = 4 * n4 + threadIdx.x; j < n; j += NT) {
      s1 += (double)PG[j] * (double)G[j];
      if (!first) s2 += (double)PG[j] * (double)Gp[j];
    }
  double v2[2] = {s1, s2};
  block_sums<2>(v2, sh);
  const double a = v2[0], b = v2[1];
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 2 + 0] = a;
    partials[blockIdx.x * 2 + 1] = b;
  }
}

__device__ __forceinline__ void f_pr_final(const double* partials, int nb, int first, DevState* st) {
  if (st->done) return;
  __shared__ double sh[SH_SUMS];
  double s2v[2];
  sum_partials_all<2>(partials, nb, sh, s2v);
  const double s1 = s2v[0], s2 = s2v[1];
  if (threadIdx.x != 0) return;
  double beta = 0.0;
  if (!first) {
    beta = (s1 - s2) / st->pg_g;
    if (!isfinite(beta)) beta = 0.0;
  }
  st->beta = beta;
  st->pg_g = s1;
}

__global__ void k_pr_final(const double* partials, int nb, int first, DevState* st) {
  f_pr_final(partials, nb, first, st);
}

template <typename T, typename TP = T>
__device__ __forceinline__ void b_direction(const TP* PG, T* D, int64_t n, int first, const DevState* st, int bid, int nb) {
  if (st->done) return;
  const double beta = st->beta;
  for (int64_t i = (int64_t)bid * NT + threadIdx.x; i < n; i += (int64_t)nb * NT) {
    const double d = first ? -(double)PG[i] : -(double)PG[i] + beta * (double)D[i];
    D[i] = (T)d;
  }
}

// One block per (K block, column tile): does the SPARSE_BN x SPARSE_BK sub-matrix hold a
// non-zero?
__global__ void k_block_pattern(const double* B, int64_t n, unsigned char* flags) {
  const int kb = blockIdx.x, t = blockIdx.y;
  const int nkb = gridDim.x;
  int nz = 0;
  for (int e = threadIdx.x; e < SPARSE_BN * SPARSE_BK; e += NT) {
    const int64_t r = (int64_t)t * SPARSE_BN + e / SPARSE_BK;
    const int64_t k = (int64_t)kb * SPARSE_BK + e % SPARSE_BK;
    if (r < n && k < n && B[r * n + k] != 0.0) nz = 1;
  }
  nz = __syncthreads_or(nz);
  if (threadIdx.x == 0) flags[(int64_t)t * nkb + kb] = (unsigned char)nz;
}

template <typename T, typename TP>
__global__ void k_direction(const TP* PG, T* D, int64_t n, int first, const DevState* st) {
  b_direction(PG, D, n, first, st, blockIdx.x, gridDim.x);
}

// The same direction rounded to bf16: D keeps the rounded values (exact in T) and `hi` their bf16
// bits (rows of length ld), so the products with D need no lo plane and the CG update moves along
// exactly this D. One row of D (rows x cols) per blockIdx.y.
template <typename T, typename TP>
__global__ void k_direction_bf16(const TP* PG, T* D, unsigned short* hi, int64_t rows, int64_t cols,
                                 int64_t ld, int first, const DevState* st) {
  if (st->done) return;
  const double beta = st->beta;
  for (int64_t r = blockIdx.y; r < rows; r += gridDim.y)
    for (int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x; c < cols;
         c += (int64_t)gridDim.x * NT) {
      const int64_t i = r * cols + c, q = r * ld + c;
      // the previous direction is exact in bf16: read back from its plane
      const double d =
          first ? -(double)PG[i]
                : -(double)PG[i] + beta * (double)__uint_as_float(((unsigned int)hi[q]) << 16);
      const unsigned short hb = bf16_bits((float)d);
      hi[q] = hb;
      if (D) D[i] = (T)__uint_as_float(((unsigned int)hb) << 16);
    }
}

// The same, four columns per thread (cols and ld multiples of 4, aligned rows) and four rows per
// block, all loads of a block's rows issued before its stores.
template <typename T, typename TP>
__global__ void k_direction_bf16x4(const TP* PG, T* D, unsigned short* hi, int64_t rows,
                                   int64_t cols, int64_t ld, int first, const DevState* st) {
  if (st->done) return;
  typedef TP P4 __attribute__((ext_vector_type(4)));
  typedef unsigned short U4 __attribute__((ext_vector_type(4)));
  constexpr int RB = 4;
  const double beta = st->beta;
  const int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (4 * c >= cols) return;
  for (int64_t r0 = (int64_t)blockIdx.y * RB; r0 < rows; r0 += (int64_t)gridDim.y * RB) {
    P4 pg[RB];
    U4 hv[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const int64_t r = r0 + k;
      if (r < rows) {
        pg[k] = *reinterpret_cast<const P4*>(PG + r * cols + 4 * c);
        if (!first) hv[k] = *reinterpret_cast<const U4*>(hi + r * ld + 4 * c);
      }
    }
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const int64_t r = r0 + k;
      if (r >= rows) continue;
      U4 h;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double prev = first ? 0.0 : (double)__uint_as_float(((unsigned int)hv[k][e]) << 16);
        const double d = first ? -(double)pg[k][e] : -(double)pg[k][e] + beta * prev;
        h[e] = bf16_bits((float)d);
      }
      *reinterpret_cast<U4*>(hi + r * ld + 4 * c) = h;
      if (D)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          D[r * cols + 4 * c + e] = (T)__uint_as_float(((unsigned int)h[e]) << 16);
    }
  }
}

// ---- quartic coefficients (Eq. 13) --------------------------------------------------------------
// Sums (index order used by the finalizer):
//  0 Tr HW   1 Tr H'   2 Tr H''
//  3 <SW,HW> 4 <S',HW> 5 <SW,H'> 6 <S'',HW> 7 <SW,H''> 8 sum S'_ij H'_ji 9 <S',H'>
//  10 <S'',H'> 11 <S',H''> 12 <S'',H''>
// With HW, SW, H'', S'' symmetric, Tr{A B} = <A, B> whenever A or B is symmetric; only
// Tr{S' H'} needs the transposed access.
__device__ __forceinline__ void b_coef_partials(const double* HW, const double* SW, const double* H1,
                                const double* S1, const double* H2, const double* S2, int M,
                                double* partials, const DevState* st, int bid, int nb) {
  if (st->done) return;
  __shared__ double t[32][33];
  __shared__ double sh[SH_SUMS];
  double acc[NCOEF];
#pragma unroll
  for (int k = 0; k < NCOEF; ++k) acc[k] = 0.0;
  const int tb = (M + 31) / 32;
  const int ntiles = tb * tb;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int tile = bid; tile < ntiles; tile += nb) {
    const int bi = (tile / tb) * 32, bj = (tile % tb) * 32;
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
      const int i = bj + r, j = bi + tx;
      t[r][tx] = (i < M && j < M) ? H1[(int64_t)i * M + j] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
      const int i = bi + r, j = bj + tx;
      if (i < M && j < M) {
        const int64_t e = (int64_t)i * M + j;
        const double hw = HW[e], sw = SW[e], h1 = H1[e], s1 = S1[e], h2 = H2[e], s2 = S2[e];
        const double h1t = t[tx][r];  // H'_ji
        if (i == j) { acc[0] += hw; acc[1] += h1; acc[2] += h2; }
        acc[3] += sw * hw;
        acc[4] += s1 * hw;
        acc[5] += sw * h1;
        acc[6] += s2 * hw;
        acc[7] += sw * h2;
        acc[8] += s1 * h1t;
        acc[9] += s1 * h1;
        acc[10] += s2 * h1;
        acc[11] += s1 * h2;
        acc[12] += s2 * h2;
      }
    }
  }
  block_sums<NCOEF>(acc, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < NCOEF; ++k) partials[bid * NCOEF + k] = acc[k];
}

__global__ void k_coef_partials(const double* HW, const double* SW, const double* H1,
                                const double* S1, const double* H2, const double* S2, int M,
                                double* partials, const DevState* st) {
  b_coef_partials(HW, SW, H1, S1, H2, S2, M, partials, st, blockIdx.x, gridDim.x);
}

// Line minimum of q(x) = sum_k a_k x^k: the first local minimum met going downhill from x = 0
// (the functional has no lower bound, so the lowest of two minima may lie beyond the basin).
// Descent side x > 0 if a1 < 0 (x < 0 if a1 > 0; a1 = 0 gives x = 0). Candidates are real roots
// of q' on that side (closed-form cubic, two Newton steps) with q'' > 0; the smallest |x| wins.
// a4 (then a3) is dropped when negligible against |a1|+|a2|+|a3|+|a4|.
__device__ double dq(const double* a, double x) {
  return a[1] + 2.0 * a[2] * x + 3.0 * a[3] * x * x + 4.0 * a[4] * x * x * x;
}
__device__ double d2q(const double* a, double x) {
  return 2.0 * a[2] + 6.0 * a[3] * x + 12.0 * a[4] * x * x;
}

__device__ int cubic_roots(double a, double b, double c, double d, double* r) {
  const double A = b / a, B = c / a, Cc = d / a;
  const double p = B - A * A / 3.0;
  const double q = 2.0 * A * A * A / 27.0 - A * B / 3.0 + Cc;
  const double sh = -A / 3.0;
  const double disc = (q / 2.0) * (q / 2.0) + (p / 3.0) * (p / 3.0) * (p / 3.0);
  if (disc > 0.0) {
    const double u = cbrt(-q / 2.0 - copysign(sqrt(disc), q));
    r[0] = u - p / (3.0 * u) + sh;
    return 1;
  }
  if (p == 0.0) {
    r[0] = sh;
    return 1;
  }
  const double m = 2.0 * sqrt(-p / 3.0);
  const double arg = fmin(1.0, fmax(-1.0, 3.0 * q / (p * m)));
  const double phi = acos(arg) / 3.0;
  const double two_pi_3 = 2.0 * M_PI / 3.0;
  for (int k = 0; k < 3; ++k) r[k] = m * cos(phi - two_pi_3 * k) + sh;
  return 3;
}

__device__ int line_minimum(const double* a, double* xout) {
  if (a[1] == 0.0) { *xout = 0.0; return 1; }
  const double side = a[1] < 0.0 ? 1.0 : -1.0;
  const double scale = fabs(a[1]) + fabs(a[2]) + fabs(a[3]) + fabs(a[4]);
  const double tiny = 1e-14 * scale;
  double roots[3];
  int nr = 0;
  if (fabs(a[4]) > tiny) {
    nr = cubic_roots(4.0 * a[4], 3.0 * a[3], 2.0 * a[2], a[1], roots);
  } else if (fabs(a[3]) > tiny) {
    const double qa = 3.0 * a[3], qb = 2.0 * a[2], qc = a[1];
    const double disc = qb * qb - 4.0 * qa * qc;
    if (disc >= 0.0) {
      const double s = -0.5 * (qb + copysign(sqrt(disc), qb));
      if (s != 0.0) roots[nr++] = qc / s;
      roots[nr++] = s / qa;
    }
  } else {
    if (a[2] > 0.0) { *xout = -a[1] / (2.0 * a[2]); return 1; }
    return 0;
  }
  int found = 0;
  double best = 0.0;
  for (int k = 0; k < nr; ++k) {
    double x = roots[k];
    for (int it = 0; it < 2; ++it) {
      const double h = d2q(a, x);
      if (h == 0.0) break;
      const double step = dq(a, x) / h;
      if (!isfinite(step)) break;
      x -= step;
    }
    if (!isfinite(x) || side * x <= 0.0 || !(d2q(a, x) > 0.0)) continue;
    if (!found || fabs(x) < fabs(best)) {
      best = x;
      found = 1;
    }
  }
  *xout = best;
  return found;
}

__device__ __forceinline__ void f_line_final(const double* partials, int nb, DevState* st) {
  if (st->done) return;
  __shared__ double sh[SH_SUMS];
  double s[NCOEF];
  sum_partials_all<NCOEF>(partials, nb, sh, s);
  if (threadIdx.x != 0) return;
  double a[5];
  a[0] = 4.0 * s[0] - 2.0 * s[3];
  a[1] = 8.0 * s[1] - 4.0 * s[4] - 4.0 * s[5];
  a[2] = 4.0 * s[2] - 2.0 * s[6] - 2.0 * s[7] - 4.0 * s[8] - 4.0 * s[9];
  a[3] = -4.0 * s[10] - 4.0 * s[11];
  a[4] = -2.0 * s[12];
  for (int k = 0; k < 5; ++k) st->alpha[k] = a[k];
  for (int k = 0; k < 5; ++k)
    if (!isfinite(a[k])) { st->done = -5; return; }
  double x = 0.0;
  if (!line_minimum(a, &x)) { st->done = -7; return; }
  st->x = x;
}

__global__ void k_line_final(const double* partials, int nb, DevState* st) {
  f_line_final(partials, nb, st);
}

// ---- updates (Eq. 16 and the footnote of Sec. 2.3) ----------------------------------------------
template <typename T, typename TD = T>
__device__ __forceinline__ void b_update_mn(T* C, const T* D, T* HC, const TD* HD, T* SC, const TD* SD, int64_t n,
                            const DevState* st, int bid, int nb) {
  if (st->done) return;
  const double x = st->x;
  for (int64_t i = (int64_t)bid * NT + threadIdx.x; i < n; i += (int64_t)nb * NT) {
    C[i] = (T)((double)C[i] + x * (double)D[i]);
    HC[i] = (T)((double)HC[i] + x * (double)HD[i]);
    SC[i] = (T)((double)SC[i] + x * (double)SD[i]);
  }
}

template <typename T, typename TD>
__global__ void k_update_mn(T* C, const T* D, T* HC, const TD* HD, T* SC, const TD* SD, int64_t n,
                            const DevState* st) {
  b_update_mn(C, D, HC, HD, SC, SD, n, st, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ void split_store(double v, unsigned short* hi, unsigned short* lo,
                                            int64_t e) {
  const unsigned short hb = bf16_bits((float)v);
  hi[e] = hb;
  lo[e] = bf16_bits((float)(v - (double)__uint_as_float(((unsigned int)hb) << 16)));
}

// Eq. 16 for C, HC, SC (rows x cols) with the bf16 planes of the new HC and SC, row-major and
// transposed (through a 32 x 33 LDS tile), one 32 x 32 tile per block.
__device__ __forceinline__ float bf16_value(unsigned short b) {
  return __uint_as_float(((unsigned int)b) << 16);
}

template <typename T, typename TD>
__global__ void k_update_split_mn(T* C, const unsigned short* Dh, int64_t ldd, T* HC, const TD* HD,
                                  T* SC, const TD* SD, int rows, int cols, StatePlanes p,
                                  const DevState* st) {
  if (st->done) return;
  __shared__ T th[32][33], ts[32][33];
  const double x = st->x;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int gr = r0 + r, gc = c0 + tx;
    T h = (T)0, v = (T)0;
    if (gr < rows && gc < cols) {
      const int64_t e = (int64_t)gr * cols + gc;
      const double d = (double)bf16_value(Dh[(int64_t)gr * ldd + gc]);
      C[e] = (T)((double)C[e] + x * d);
      h = (T)((double)HC[e] + x * (double)HD[e]);
      v = (T)((double)SC[e] + x * (SD ? (double)SD[e] : d));
      HC[e] = h;
      SC[e] = v;
      const int64_t q = (int64_t)gr * p.ld + gc;
      split_store((double)h, p.hc_hi, p.hc_lo, q);
      split_store((double)v, p.sc_hi, p.sc_lo, q);
    }
    th[r][tx] = h;
    ts[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int oc = c0 + r, orow = r0 + tx;  // output row oc (a source column), column orow
    if (oc < cols && orow < rows) {
      const int64_t o = (int64_t)oc * p.ldt + orow;
      split_store((double)th[tx][r], p.hct_hi, p.hct_lo, o);
      split_store((double)ts[tx][r], p.sct_hi, p.sct_lo, o);
    }
  }
}

// The same for an even number of columns (8-byte aligned rows), one 64 x 64 tile per block:
// each thread takes two adjacent columns, so the T arrays move in 16-byte and the planes in
// 4-byte (two bf16) accesses, and every plane row segment a block writes (also transposed) is
// one 128-byte line. The transpose goes through LDS as packed (hi | lo << 16) words. Every store
// is non-temporal (see stream_store).
__device__ __forceinline__ unsigned split_word(double v) {
  const unsigned hb = bf16_bits((float)v);
  const unsigned lb = bf16_bits((float)(v - (double)__uint_as_float(hb << 16)));
  return hb | (lb << 16);
}

// Two bf16 values as one 4-byte store that bypasses the caches' normal retention: everything
// the update writes is next read a whole line search later, long after it would have left L2.
__device__ __forceinline__ void stream_store(unsigned w, unsigned short* dst) {
  __builtin_nontemporal_store(w, reinterpret_cast<unsigned*>(dst));
}

template <typename T, typename TD>
__global__ __launch_bounds__(NT) void k_update_split_mn2(T* C, const unsigned short* Dh,
                                                         int64_t ldd, T* HC, const TD* HD, T* SC,
                                                         const TD* SD, int rows, int cols,
                                                         StatePlanes p, const DevState* st) {
  if (st->done) return;
  typedef T T2 __attribute__((ext_vector_type(2)));
  typedef TD TD2 __attribute__((ext_vector_type(2)));
  __shared__ unsigned th[64][65], ts[64][65];
  const double x = st->x;
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 column pairs x 8 rows
  const int gc = c0 + 2 * tx;
  // rows ty + 8 k, four at a time: all loads of a batch are issued before its stores
  constexpr int RB = 4;
#pragma unroll
  for (int b = 0; b < 8; b += RB) {
    T2 c[RB], hc[RB], sc[RB];
    TD2 hd[RB], sd[RB];
    unsigned dw[RB];  // two bf16 directions
    bool in[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const int gr = r0 + ty + 8 * (b + k);
      in[k] = gr < rows && gc < cols;  // cols even: gc + 1 < cols as well
      if (in[k]) {
        const int64_t e = (int64_t)gr * cols + gc;
        c[k] = *reinterpret_cast<const T2*>(C + e);
        dw[k] = *reinterpret_cast<const unsigned*>(Dh + (int64_t)gr * ldd + gc);
        hc[k] = *reinterpret_cast<const T2*>(HC + e);
        hd[k] = *reinterpret_cast<const TD2*>(HD + e);
        sc[k] = *reinterpret_cast<const T2*>(SC + e);
        if (SD) sd[k] = *reinterpret_cast<const TD2*>(SD + e);
      }
    }
#pragma unroll
    for (int k = 0; k < RB; ++k) {
      const int r = ty + 8 * (b + k), gr = r0 + r;
      unsigned wh0 = 0, wh1 = 0, ws0 = 0, ws1 = 0;
      if (in[k]) {
        const int64_t e = (int64_t)gr * cols + gc;
        const double d0 = (double)__uint_as_float(dw[k] << 16);
        const double d1 = (double)__uint_as_float(dw[k] & 0xffff0000u);
        T2 cn, h, v;
        cn.x = (T)((double)c[k].x + x * d0);
        cn.y = (T)((double)c[k].y + x * d1);
        h.x = (T)((double)hc[k].x + x * (double)hd[k].x);
        h.y = (T)((double)hc[k].y + x * (double)hd[k].y);
        v.x = (T)((double)sc[k].x + x * (SD ? (double)sd[k].x : d0));
        v.y = (T)((double)sc[k].y + x * (SD ? (double)sd[k].y : d1));
        __builtin_nontemporal_store(cn, reinterpret_cast<T2*>(C + e));
        __builtin_nontemporal_store(h, reinterpret_cast<T2*>(HC + e));
        __builtin_nontemporal_store(v, reinterpret_cast<T2*>(SC + e));
        wh0 = split_word((double)h.x);
        wh1 = split_word((double)h.y);
        ws0 = split_word((double)v.x);
        ws1 = split_word((double)v.y);
        const int64_t q = (int64_t)gr * p.ld + gc;
        stream_store((wh0 & 0xffffu) | (wh1 << 16), p.hc_hi + q);
        stream_store((wh0 >> 16) | (wh1 & 0xffff0000u), p.hc_lo + q);
        stream_store((ws0 & 0xffffu) | (ws1 << 16), p.sc_hi + q);
        stream_store((ws0 >> 16) | (ws1 & 0xffff0000u), p.sc_lo + q);
      }
      th[r][2 * tx] = wh0;
      th[r][2 * tx + 1] = wh1;
      ts[r][2 * tx] = ws0;
      ts[r][2 * tx + 1] = ws1;
    }
  }
  __syncthreads();
  // transposed: output row oc = c0 + j (a source column), output columns r0 + 2 tx, r0 + 2 tx + 1
  const int orow = r0 + 2 * tx;
  for (int j = ty; j < 64; j += 8) {
    const int oc = c0 + j;
    if (oc >= cols || orow >= rows) continue;
    const unsigned a0 = th[2 * tx][j], b0 = ts[2 * tx][j];
    const int64_t o = (int64_t)oc * p.ldt + orow;
    if (orow + 1 < rows) {
      const unsigned a1 = th[2 * tx + 1][j], b1 = ts[2 * tx + 1][j];
      stream_store((a0 & 0xffffu) | (a1 << 16), p.hct_hi + o);
      stream_store((a0 >> 16) | (a1 & 0xffff0000u), p.hct_lo + o);
      stream_store((b0 & 0xffffu) | (b1 << 16), p.sct_hi + o);
      stream_store((b0 >> 16) | (b1 & 0xffff0000u), p.sct_lo + o);
    } else {
      p.hct_hi[o] = (unsigned short)(a0 & 0xffffu);
      p.hct_lo[o] = (unsigned short)(a0 >> 16);
      p.sct_hi[o] = (unsigned short)(b0 & 0xffffu);
      p.sct_lo[o] = (unsigned short)(b0 >> 16);
    }
  }
}

// Real embedding of a complex matrix Z (rows 2 rh): row rh + r is the pair rotation of row r,
// [-Im z, Re z] for [Re z, Im z] (each half h columns). Products whose rows follow the row pairs
// of C are computed for the first rh rows; this fills the others, and the same rotation of the
// optional bf16 planes (negation flips the sign bit: bf16 rounding is symmetric).
template <typename T>
__global__ void k_pair_rows(T* X, int64_t ld, unsigned short* hi, unsigned short* lo, int64_t ldp,
                            int rh, int h, const DevState* st) {
  if (st && st->done) return;
  for (int64_t r = blockIdx.y; r < rh; r += gridDim.y)
    for (int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x; c < 2 * (int64_t)h;
         c += (int64_t)gridDim.x * NT) {
      const bool neg = c < h;
      const int64_t src = neg ? c + h : c - h;
      const T v = X[r * ld + src];
      X[(r + rh) * ld + c] = neg ? -v : v;
      if (hi) {
        const unsigned short sgn = neg ? 0x8000 : 0;
        hi[(r + rh) * ldp + c] = hi[r * ldp + src] ^ sgn;
        lo[(r + rh) * ldp + c] = lo[r * ldp + src] ^ sgn;
      }
    }
}

// HW += x (H' + H'^T) + x^2 H'', SW likewise; partial sums of Tr HW, <SW, HW>, Tr SW.
__device__ __forceinline__ void b_update_mm(double* HW, double* SW, const double* H1, const double* S1,
                            const double* H2, const double* S2, int M, double* partials,
                            const DevState* st, int bid, int nb) {
  if (st->done) return;
  __shared__ double th[32][33], ts[32][33];
  __shared__ double sh[SH_SUMS];
  const double x = st->x;
  double tr = 0.0, f = 0.0, trs = 0.0;
  const int tb = (M + 31) / 32;
  const int ntiles = tb * tb;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int tile = bid; tile < ntiles; tile += nb) {
    const int bi = (tile / tb) * 32, bj = (tile % tb) * 32;
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
      const int i = bj + r, j = bi + tx;
      const bool in = i < M && j < M;
      th[r][tx] = in ? H1[(int64_t)i * M + j] : 0.0;
      ts[r][tx] = in ? S1[(int64_t)i * M + j] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
      const int i = bi + r, j = bj + tx;
      if (i < M && j < M) {
        const int64_t e = (int64_t)i * M + j;
        const double hw = HW[e] + x * H1[e] + x * th[tx][r] + x * x * H2[e];
        const double sw = SW[e] + x * S1[e] + x * ts[tx][r] + x * x * S2[e];
        HW[e] = hw;
        SW[e] = sw;
        f += sw * hw;
        if (i == j) { tr += hw; trs += sw; }
      }
    }
  }
  double v3[3] = {tr, f, trs};
  block_sums<3>(v3, sh);
  const double a = v3[0], b = v3[1], c = v3[2];
  if (threadIdx.x == 0) {
    partials[bid * 3 + 0] = a;
    partials[bid * 3 + 1] = b;
    partials[bid * 3 + 2] = c;
  }
}

// The same update for one system, using that HW, SW, H'' and S'' are symmetric: each block takes a
// pair of 32 x 32 tiles (bi, bj), bi <= bj, computes the upper one from the upper tiles of HW,
// SW, H'', S'' and both tiles of H', S' (the mirror one transposed through LDS), and writes the
// result to both (on a diagonal tile, its upper triangle to both halves). HW and SW come out
// exactly symmetric; every element of H', S' and of the upper halves is read once.
__global__ __launch_bounds__(NT) void k_update_mm_sym(double* HW, double* SW, const double* H1,
                                                      const double* S1, const double* H2,
                                                      const double* S2, int M, double* partials,
                                                      const DevState* st) {
  if (st->done) return;
  __shared__ double th[32][33], ts[32][33], oh[32][33], os[32][33];
  __shared__ double sh[SH_SUMS];
  const double x = st->x;
  double tr = 0.0, f = 0.0, trs = 0.0;
  const int T = (M + 31) / 32;
  const int npairs = T * (T + 1) / 2;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int p = blockIdx.x; p < npairs; p += gridDim.x) {
    int bi = 0, rem = p;
    while (rem >= T - bi) {
      rem -= T - bi;
      ++bi;
    }
    const int bj = bi + rem;
    const int i0 = bi * 32, j0 = bj * 32;
    const bool diag = bi == bj;
    __syncthreads();
    // th[c][r] = H'[j0 + c][i0 + r], the transposed partner of output (i0 + r, j0 + c)
    for (int rr = ty; rr < 32; rr += 8) {
      const int i = j0 + rr, j = i0 + tx;
      const bool in = i < M && j < M;
      th[rr][tx] = in ? H1[(int64_t)i * M + j] : 0.0;
      ts[rr][tx] = in ? S1[(int64_t)i * M + j] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
      const int i = i0 + r, j = j0 + tx;
      if (i < M && j < M && (!diag || r <= tx)) {
        const int64_t e = (int64_t)i * M + j;
        const double hw = HW[e] + x * H1[e] + x * th[tx][r] + x * x * H2[e];
        const double sw = SW[e] + x * S1[e] + x * ts[tx][r] + x * x * S2[e];
        HW[e] = hw;
        SW[e] = sw;
        oh[r][tx] = hw;
        os[r][tx] = sw;
        if (diag && r == tx) {
          tr += hw;
          trs += sw;
          f += sw * hw;
        } else {
          f += 2.0 * sw * hw;
        }
      }
    }
    __syncthreads();
    // mirror: element (j0 + rr, i0 + tx) = output (i0 + tx, j0 + rr)
    for (int rr = ty; rr < 32; rr += 8) {
      const int i = j0 + rr, j = i0 + tx;
      if (i < M && j < M && (!diag || tx < rr)) {
        const int64_t e = (int64_t)i * M + j;
        HW[e] = oh[tx][rr];
        SW[e] = os[tx][rr];
      }
    }
  }
  double v3[3] = {tr, f, trs};
  block_sums<3>(v3, sh);
  const double a = v3[0], b = v3[1], c = v3[2];
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 3 + 0] = a;
    partials[blockIdx.x * 3 + 1] = b;
    partials[blockIdx.x * 3 + 2] = c;
  }
}

__device__ __forceinline__ void f_update_final(const double* partials, int nb, int M, DevState* st,
                               double* trace) {
  if (st->done) return;
  __shared__ double sh[SH_SUMS];
  double s3[3];
  sum_partials_all<3>(partials, nb, sh, s3);
  const double tr = s3[0], f = s3[1], trs = s3[2];
  if (threadIdx.x != 0) return;
  const double E_new = 4.0 * tr - 2.0 * f;
  const double E_old = st->E;
  const double diff = fabs(2.0 * (E_new - E_old)), sum = fabs(E_new + E_old);
  st->E_prev = E_old;
  st->E = E_new;
  st->iter += 1;
  st->rel_change = sum > 0.0 ? diff / sum : diff;
  if (trace) trace[st->iter] = E_new;
  if (!isfinite(E_new)) { st->done = -5; return; }
  if (trs > 16.0 * (double)M) { st->done = -8; return; }
  if (diff <= st->tol * sum) { st->done = 1; return; }
  if (st->iter >= st->max_iter) st->done = 2;
}

__global__ void k_update_final(const double* partials, int nb, int M, DevState* st,
                               double* trace) {
  f_update_final(partials, nb, M, st, trace);
}

__global__ void k_identity_minus(const double* SW, double* out, int M, double diag, double scale) {
  const int64_t n = (int64_t)M * M;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    const int r = (int)(i / M), c = (int)(i % M);
    out[i] = scale * ((r == c ? diag : 0.0) - SW[i]);
  }
}

__global__ void k_axpby(const double* a, const double* b, double* out, double ca, double cb,
                        int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    out[i] = ca * a[i] + cb * b[i];
}

__global__ void k_scale(double* a, double c, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
    a[i] *= c;
}

// ---- grouped kernels (blockIdx.y = system) -----------------------------------------------------
__global__ void g_energy_partials(const SysDev* sys) {
  const SysDev& d = sys[blockIdx.y];
  b_energy_partials(d.HW, d.SW, d.M, d.partials, blockIdx.x, gridDim.x);
}
__global__ void g_energy_init_final(const SysDev* sys) {
  const SysDev& d = sys[blockIdx.y];
  f_energy_init_final(d.partials, GROUP_BLOCKS, d.st, d.trace);
}
template <typename T>
__device__ __forceinline__ void g_pr_partials_t(const SysDev& d, int parity, int first) {
  const T* G = static_cast<const T*>(parity ? d.G1 : d.G0);
  const T* Gp = static_cast<const T*>(parity ? d.G0 : d.G1);
  const T* PG = d.precon ? static_cast<const T*>(d.PG) : G;
  b_pr_partials<T>(G, PG, Gp, (int64_t)d.M * d.N, first, d.partials, d.st, blockIdx.x, gridDim.x);
}
__global__ void g_pr_partials(const SysDev* sys, int parity, int first) {
  const SysDev& d = sys[blockIdx.y];
  if (d.f64) g_pr_partials_t<double>(d, parity, first);
  else g_pr_partials_t<float>(d, parity, first);
}
__global__ void g_pr_final(const SysDev* sys, int first) {
  const SysDev& d = sys[blockIdx.y];
  f_pr_final(d.partials, GROUP_BLOCKS, first, d.st);
}
template <typename T>
__device__ __forceinline__ void g_direction_t(const SysDev& d, int parity, int first) {
  const T* G = static_cast<const T*>(parity ? d.G1 : d.G0);
  const T* PG = d.precon ? static_cast<const T*>(d.PG) : G;
  b_direction<T>(PG, static_cast<T*>(d.D), (int64_t)d.M * d.N, first, d.st, blockIdx.x,
                 gridDim.x);
}
__global__ void g_direction(const SysDev* sys, int parity, int first) {
  const SysDev& d = sys[blockIdx.y];
  if (d.f64) g_direction_t<double>(d, parity, first);
  else g_direction_t<float>(d, parity, first);
}
__global__ void g_coef_partials(const SysDev* sys) {
  const SysDev& d = sys[blockIdx.y];
  b_coef_partials(d.HW, d.SW, d.H1, d.S1, d.H2, d.S2, d.M, d.partials, d.st, blockIdx.x, gridDim.x);
}
__global__ void g_line_final(const SysDev* sys) {
  const SysDev& d = sys[blockIdx.y];
  f_line_final(d.partials, GROUP_BLOCKS, d.st);
}
template <typename T>
__device__ __forceinline__ void g_update_mn_t(const SysDev& d) {
  b_update_mn<T>(static_cast<T*>(d.C), static_cast<const T*>(d.D), static_cast<T*>(d.HC),
                 static_cast<const T*>(d.HD), static_cast<T*>(d.SC), static_cast<const T*>(d.SD),
                 (int64_t)d.M * d.N, d.st, blockIdx.x, gridDim.x);
}
__global__ void g_update_mn(const SysDev* sys) {
  const SysDev& d = sys[blockIdx.y];
  if (d.f64) g_update_mn_t<double>(d);
  else g_update_mn_t<float>(d);
}
template <typename T>
__device__ __forceinline__ void pair_fill(T* X, int rh, int h, int64_t r, int64_t c) {
  const bool neg = c < h;
  const T v = X[r * 2 * h + (neg ? c + h : c - h)];
  X[(r + rh) * 2 * h + c] = neg ? -v : v;
}

__global__ void g_pair_rows(const SysDev* sys, int which, int parity, int check_done) {
  const SysDev& d = sys[blockIdx.z];
  if (!d.paired || (check_done && d.st->done)) return;
  if (which == 3 && !d.precon) return;  // PG aliases G
  const int rh = d.M / 2;
  const bool mm = which == 1 || which == 5;  // M x M (FP64) or M x N (FP32 or FP64 state)
  const int h = (mm ? d.M : d.N) / 2;
  void* xs[2] = {nullptr, nullptr};  // M x N arrays of the state's type
  double* xd[4] = {nullptr, nullptr, nullptr, nullptr};
  if (which == 0) { xs[0] = d.HC; xs[1] = d.SC; }
  if (which == 2) xs[0] = parity ? d.G1 : d.G0;
  if (which == 3) xs[0] = d.PG;
  if (which == 4) { xs[0] = d.HD; xs[1] = d.SD; }
  if (which == 1) { xd[0] = d.HW; xd[1] = d.SW; }
  if (which == 5) { xd[0] = d.H1; xd[1] = d.S1; xd[2] = d.H2; xd[3] = d.S2; }
  for (int64_t r = blockIdx.y; r < rh; r += gridDim.y)
    for (int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x; c < 2 * (int64_t)h;
         c += (int64_t)gridDim.x * NT) {
      for (int a = 0; a < 2; ++a) {
        if (!xs[a]) continue;
        if (d.f64) pair_fill(static_cast<double*>(xs[a]), rh, h, r, c);
        else pair_fill(static_cast<float*>(xs[a]), rh, h, r, c);
      }
      for (int a = 0; a < 4; ++a)
        if (xd[a]) pair_fill(xd[a], rh, h, r, c);
    }
}

__global__ void g_update_mm(const SysDev* sys) {
  const SysDev& d = sys[blockIdx.y];
  b_update_mm(d.HW, d.SW, d.H1, d.S1, d.H2, d.S2, d.M, d.partials, d.st, blockIdx.x, gridDim.x);
}
__global__ void g_update_final(const SysDev* sys) {
  const SysDev& d = sys[blockIdx.y];
  f_update_final(d.partials, GROUP_BLOCKS, d.M, d.st, d.trace);
}

int tile_blocks(int M) {
  const int tb = (M + 31) / 32;
  int b = tb * tb;
  return b > RED_BLOCKS ? RED_BLOCKS : b;
}

}  // namespace

hipError_t shift_hamiltonian(const double* H, const double* S, double eta, double* Hs, int64_t n,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_shift, dim3(ew_blocks(n)), dim3(NT), 0, s, H, S, eta, Hs, n);
  return hipGetLastError();
}

hipError_t convert_f64_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<double, float>), dim3(ew_blocks(n)), dim3(NT), 0, s, src, dst, n);
  return hipGetLastError();
}

namespace {
dim3 split_grid(int64_t rows, int64_t cols) {
  int64_t bx = (cols + 4 * NT - 1) / (4 * NT);
  if (bx < 1) bx = 1;
  return dim3((unsigned)bx, (unsigned)(rows < 65535 ? rows : 65535));
}
}  // namespace

hipError_t split_bf16(const float* src, unsigned short* hi, unsigned short* lo, int64_t rows,
                      int64_t cols, int64_t ld, const DevState* st, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (ld < cols || ld % 4 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_split<float>, split_grid(rows, cols), dim3(NT), 0, s, src, hi, lo, rows, cols,
                     ld, st);
  return hipGetLastError();
}

hipError_t split_bf16(const double* src, unsigned short* hi, unsigned short* lo, int64_t rows,
                      int64_t cols, int64_t ld, const DevState* st, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (ld < cols || ld % 4 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_split<double>, split_grid(rows, cols), dim3(NT), 0, s, src, hi, lo, rows,
                     cols, ld, st);
  return hipGetLastError();
}

hipError_t split_bf16_t(const float* src, unsigned short* hi, unsigned short* lo, int rows,
                        int cols, int64_t ld, const DevState* st, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (ld < rows) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_split_t<float>, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(NT), 0, s, src,
                     hi, lo, rows, cols, ld, st);
  return hipGetLastError();
}

hipError_t split_bf16_t(const double* src, unsigned short* hi, unsigned short* lo, int rows,
                        int cols, int64_t ld, const DevState* st, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (ld < rows) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_split_t<double>, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(NT), 0, s,
                     src, hi, lo, rows, cols, ld, st);
  return hipGetLastError();
}

hipError_t pair_rows(void* X, bool f64, int64_t ld, unsigned short* hi, unsigned short* lo,
                     int64_t ldp, int rh, int h, const DevState* st, hipStream_t s) {
  if (rh <= 0 || h <= 0) return hipSuccess;
  if (ld < 2 * (int64_t)h || (hi && (!lo || ldp < 2 * (int64_t)h))) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((2 * (int64_t)h + NT - 1) / NT), (unsigned)(rh < 65535 ? rh : 65535));
  if (f64)
    hipLaunchKernelGGL(k_pair_rows<double>, grid, dim3(NT), 0, s, static_cast<double*>(X), ld, hi,
                       lo, ldp, rh, h, st);
  else
    hipLaunchKernelGGL(k_pair_rows<float>, grid, dim3(NT), 0, s, static_cast<float*>(X), ld, hi, lo,
                       ldp, rh, h, st);
  return hipGetLastError();
}

hipError_t convert_f32_f64(const float* src, double* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<float, double>), dim3(ew_blocks(n)), dim3(NT), 0, s, src, dst, n);
  return hipGetLastError();
}

// dst = src; *diff = 1 if any element changes (bit pattern), else *diff is left as it was
__global__ void k_copy_compare(const double* src, double* dst, int64_t n, int* diff) {
  bool changed = false;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    const double v = src[i];
    changed |= __double_as_longlong(v) != __double_as_longlong(dst[i]);
    dst[i] = v;
  }
  if (__any(changed) && (threadIdx.x & 63) == 0) atomicOr(diff, 1);
}

hipError_t copy_compare_f64(const double* src, double* dst, int64_t n, int* diff, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_compare, dim3(ew_blocks(n)), dim3(NT), 0, s, src, dst, n, diff);
  return hipGetLastError();
}

hipError_t copy_f64(const double* src, double* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<double, double>), dim3(ew_blocks(n)), dim3(NT), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t validate_symmetric(const double* A, int64_t n, double rtol, int* flags, hipStream_t s) {
  const int tb = (int)((n + 31) / 32);
  hipLaunchKernelGGL(k_validate, dim3(tb, tb), dim3(NT), 0, s, A, n, rtol, flags);
  return hipGetLastError();
}

hipError_t symmetrize(double* A, int64_t n, hipStream_t s) {
  const int tb = (int)((n + 31) / 32);
  hipLaunchKernelGGL(k_symmetrize, dim3(tb, tb), dim3(NT), 0, s, A, n);
  return hipGetLastError();
}

hipError_t energy_init(const double* HW, const double* SW, int M, double* partials, DevState* st,
                       double* trace, hipStream_t s) {
  const int nb = red_blocks((int64_t)M * M);
  hipLaunchKernelGGL(k_energy_partials, dim3(nb), dim3(NT), 0, s, HW, SW, M, partials);
  hipLaunchKernelGGL(k_energy_init_final, dim3(1), dim3(NT), 0, s, partials, nb, st, trace);
  return hipGetLastError();
}

hipError_t block_pattern(const double* B, int64_t n, unsigned char* flags, hipStream_t s) {
  const int nkb = (int)((n + SPARSE_BK - 1) / SPARSE_BK);
  const int nt = (int)((n + SPARSE_BN - 1) / SPARSE_BN);
  hipLaunchKernelGGL(k_block_pattern, dim3(nkb, nt), dim3(NT), 0, s, B, n, flags);
  return hipGetLastError();
}

template <typename T, typename TP, typename TG>
hipError_t beta_and_direction(const TG* G, const TP* PG, const TG* Gprev, T* D, int64_t n, int first,
                              double* partials, DevState* st, hipStream_t s, unsigned short* hi,
                              int64_t cols, int64_t ld) {
  if (!hi && !D) return hipErrorInvalidValue;
  const int nb = red_blocks(n);
  const bool vec = ((uintptr_t)G | (uintptr_t)Gprev) % (4 * sizeof(TG)) == 0 &&
                   (uintptr_t)PG % (4 * sizeof(TP)) == 0;
  if (vec)
    hipLaunchKernelGGL((k_pr_partials4<TG, TP>), dim3(nb), dim3(NT), 0, s, G, PG, Gprev, n, first,
                       partials, st);
  else
    hipLaunchKernelGGL((k_pr_partials<TG, TP>), dim3(nb), dim3(NT), 0, s, G, PG, Gprev, n, first,
                       partials, st);
  hipLaunchKernelGGL(k_pr_final, dim3(1), dim3(NT), 0, s, partials, nb, first, st);
  if (hi) {
    if (cols <= 0 || n % cols != 0 || ld < cols) return hipErrorInvalidValue;
    const int64_t rows = n / cols;
    const bool vec4 = cols % 4 == 0 && ld % 4 == 0 && (uintptr_t)PG % (4 * sizeof(TP)) == 0 &&
                      (uintptr_t)hi % 8 == 0;
    if (vec4) {
      const int64_t bx = (cols / 4 + NT - 1) / NT, by = (rows + 3) / 4;
      hipLaunchKernelGGL((k_direction_bf16x4<T, TP>), dim3((unsigned)bx, (unsigned)(by < 65535 ? by : 65535)),
                         dim3(NT), 0, s, PG, D, hi, rows, cols, ld, first, st);
    } else {
      const int64_t bx = (cols + NT - 1) / NT;
      hipLaunchKernelGGL((k_direction_bf16<T, TP>), dim3((unsigned)bx, (unsigned)(rows < 65535 ? rows : 65535)),
                         dim3(NT), 0, s, PG, D, hi, rows, cols, ld, first, st);
    }
  } else {
    hipLaunchKernelGGL((k_direction<T, TP>), dim3(ew_blocks(n)), dim3(NT), 0, s, PG, D, n, first, st);
  }
  return hipGetLastError();
}
#define OMM_BETA_DIRECTION(T, TP, TG)                                                            \
  template hipError_t beta_and_direction<T, TP, TG>(const TG*, const TP*, const TG*, T*, int64_t, \
                                                    int, double*, DevState*, hipStream_t,         \
                                                    unsigned short*, int64_t, int64_t);
OMM_BETA_DIRECTION(double, double, double)
OMM_BETA_DIRECTION(float, float, float)
OMM_BETA_DIRECTION(double, float, double)
OMM_BETA_DIRECTION(double, float, float)
#undef OMM_BETA_DIRECTION

hipError_t line_search(const double* HW, const double* SW, const double* H1, const double* S1,
                       const double* H2, const double* S2, int M, double* partials, DevState* st,
                       hipStream_t s) {
  const int nb = tile_blocks(M);
  hipLaunchKernelGGL(k_coef_partials, dim3(nb), dim3(NT), 0, s, HW, SW, H1, S1, H2, S2, M,
                     partials, st);
  hipLaunchKernelGGL(k_line_final, dim3(1), dim3(NT), 0, s, partials, nb, st);
  return hipGetLastError();
}

template <typename T, typename TD>
hipError_t update_coefficients(T* C, const T* D, T* HC, const TD* HD, T* SC, const TD* SD,
                               int64_t n, const DevState* st, hipStream_t s) {
  hipLaunchKernelGGL((k_update_mn<T, TD>), dim3(ew_blocks(n)), dim3(NT), 0, s, C, D, HC, HD, SC, SD,
                     n, st);
  return hipGetLastError();
}
#define OMM_UPDATE(T, TD)                                                                        \
  template hipError_t update_coefficients<T, TD>(T*, const T*, T*, const TD*, T*, const TD*,     \
                                                 int64_t, const DevState*, hipStream_t);
OMM_UPDATE(double, double)
OMM_UPDATE(float, float)
OMM_UPDATE(double, float)
#undef OMM_UPDATE

template <typename T, typename TD>
hipError_t update_coefficients_split(T* C, const unsigned short* Dh, int64_t ldd, T* HC,
                                     const TD* HD, T* SC, const TD* SD, int rows, int cols,
                                     const StatePlanes& p, const DevState* st, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (!Dh || ldd < cols || p.ld < cols || p.ldt < rows) return hipErrorInvalidValue;
  const bool wide = cols % 2 == 0 && p.ld % 2 == 0 && p.ldt % 2 == 0 && ldd % 2 == 0 &&
                    (uintptr_t)Dh % 4 == 0 &&
                    ((uintptr_t)C | (uintptr_t)HC | (uintptr_t)SC) % (2 * sizeof(T)) == 0 &&
                    ((uintptr_t)HD | (uintptr_t)SD) % (2 * sizeof(TD)) == 0;
  if (wide)
    hipLaunchKernelGGL((k_update_split_mn2<T, TD>), dim3((cols + 63) / 64, (rows + 63) / 64),
                       dim3(NT), 0, s, C, Dh, ldd, HC, HD, SC, SD, rows, cols, p, st);
  else
    hipLaunchKernelGGL((k_update_split_mn<T, TD>), dim3((cols + 31) / 32, (rows + 31) / 32),
                       dim3(NT), 0, s, C, Dh, ldd, HC, HD, SC, SD, rows, cols, p, st);
  return hipGetLastError();
}
#define OMM_UPDATE_SPLIT(T, TD)                                                                  \
  template hipError_t update_coefficients_split<T, TD>(T*, const unsigned short*, int64_t, T*,   \
                                                       const TD*, T*, const TD*, int, int,       \
                                                       const StatePlanes&, const DevState*,      \
                                                       hipStream_t);
OMM_UPDATE_SPLIT(double, double)
OMM_UPDATE_SPLIT(float, float)
OMM_UPDATE_SPLIT(double, float)
#undef OMM_UPDATE_SPLIT

hipError_t update_subspace(double* HW, double* SW, const double* H1, const double* S1,
                           const double* H2, const double* S2, int M, double* partials,
                           DevState* st, double* trace, hipStream_t s) {
  const int T = (M + 31) / 32, npairs = T * (T + 1) / 2;
  const int nb = npairs < RED_BLOCKS ? npairs : RED_BLOCKS;
  hipLaunchKernelGGL(k_update_mm_sym, dim3(nb), dim3(NT), 0, s, HW, SW, H1, S1, H2, S2, M, partials,
                     st);
  hipLaunchKernelGGL(k_update_final, dim3(1), dim3(NT), 0, s, partials, nb, M, st, trace);
  return hipGetLastError();
}

hipError_t group_energy_init(const SysDev* d_sys, int nsys, hipStream_t s) {
  hipLaunchKernelGGL(g_energy_partials, dim3(GROUP_BLOCKS, nsys), dim3(NT), 0, s, d_sys);
  hipLaunchKernelGGL(g_energy_init_final, dim3(1, nsys), dim3(NT), 0, s, d_sys);
  return hipGetLastError();
}

hipError_t group_direction(const SysDev* d_sys, int nsys, int parity, int first, hipStream_t s) {
  hipLaunchKernelGGL(g_pr_partials, dim3(GROUP_BLOCKS, nsys), dim3(NT), 0, s, d_sys, parity, first);
  hipLaunchKernelGGL(g_pr_final, dim3(1, nsys), dim3(NT), 0, s, d_sys, first);
  hipLaunchKernelGGL(g_direction, dim3(4 * GROUP_BLOCKS, nsys), dim3(NT), 0, s, d_sys, parity, first);
  return hipGetLastError();
}

hipError_t group_line_search(const SysDev* d_sys, int nsys, hipStream_t s) {
  hipLaunchKernelGGL(g_coef_partials, dim3(GROUP_BLOCKS, nsys), dim3(NT), 0, s, d_sys);
  hipLaunchKernelGGL(g_line_final, dim3(1, nsys), dim3(NT), 0, s, d_sys);
  return hipGetLastError();
}

hipError_t group_update(const SysDev* d_sys, int nsys, hipStream_t s) {
  hipLaunchKernelGGL(g_update_mn, dim3(4 * GROUP_BLOCKS, nsys), dim3(NT), 0, s, d_sys);
  hipLaunchKernelGGL(g_update_mm, dim3(GROUP_BLOCKS, nsys), dim3(NT), 0, s, d_sys);
  hipLaunchKernelGGL(g_update_final, dim3(1, nsys), dim3(NT), 0, s, d_sys);
  return hipGetLastError();
}

hipError_t group_pair_rows(const SysDev* d_sys, int nsys, int which, int parity, bool check_done,
                           int max_m, int max_n, hipStream_t s) {
  if (nsys <= 0 || max_m < 2) return hipSuccess;
  const int cols = (which == 1 || which == 5) ? max_m : max_n;
  const dim3 grid((unsigned)((cols + NT - 1) / NT), (unsigned)std::min(max_m / 2, 4096),
                  (unsigned)nsys);
  hipLaunchKernelGGL(g_pair_rows, grid, dim3(NT), 0, s, d_sys, which, parity, check_done ? 1 : 0);
  return hipGetLastError();
}

hipError_t identity_minus(const double* SW, double* out, int M, double diag, double scale,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_identity_minus, dim3(ew_blocks((int64_t)M * M)), dim3(NT), 0, s, SW, out, M,
                     diag, scale);
  return hipGetLastError();
}

hipError_t axpby_f64(const double* a, const double* b, double* out, double ca, double cb, int64_t n,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(ew_blocks(n)), dim3(NT), 0, s, a, b, out, ca, cb, n);
  return hipGetLastError();
}

hipError_t scale_f64(double* a, double c, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(ew_blocks(n)), dim3(NT), 0, s, a, c, n);
  return hipGetLastError();
}

}  // namespace omm
