// One-time FP64 inversion for the preconditioner P = (S + T/tau)^-1 (Sec. 2.4, Eq. 17): an
// in-place blocked Gauss-Jordan sweep. The paper inverts once per MD step with a library
// LU, since P need not be positive definite (Sec. 3.1); here each block column costs one
// pivot-block inversion plus two MFMA GEMMs, so the 2 n^3 flops run on matrix cores.
//
// Step for pivot block K (width b), with A the current matrix:
//   U  = A[:, K] with its diagonal block replaced by A_KK - I      (column panel copy)
//   W  = A_KK^-1                                                    (one workgroup, in LDS)
//   A[:, K] = e_K  (zero column panel, identity diagonal block)
//   R  = W A[K, :]                                                  (b x n GEMM)
//   A -= U R                                                        (rank-b GEMM update)
// which leaves A[K,K] = W, A[K,J] = W A_KJ, A[I,K] = -A_IK W and the Schur update elsewhere;
// after the last block A holds the inverse. The pivot block is inverted by Gauss-Jordan with
// partial (row) pivoting inside the block, so an indefinite S + T/tau whose diagonal entries
// vanish or change sign along the sweep is handled as long as each pivot block is
// nonsingular; the blocks themselves are not exchanged. A singular pivot block or a non-finite
// value is reported, and inverse_residual() measures ||A P X - X|| on probe vectors so that a
// caller can reject an inaccurate inverse instead of using it.
#include <math.h>

#include "omm_internal.h"

namespace omm {
namespace {

constexpr int NB = 128;
constexpr int PROBES = 16;  // probe rows of inverse_residual

// U = A[:, k0:k0+b] (ld b) with U[k0+i][i] -= 1; W = A[k0:k0+b, k0:k0+b]; then
// A[:, k0:k0+b] = e_K.
__global__ void k_panel(double* A, int64_t n, int64_t k0, int b, double* U, double* W) {
  const int64_t total = n * b;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / b;
    const int j = (int)(e % b);
    const double v = A[i * n + k0 + j];
    const bool diag_blk = i >= k0 && i < k0 + b;
    U[e] = (diag_blk && i - k0 == j) ? v - 1.0 : v;
    if (diag_blk) W[(i - k0) * b + j] = v;
    A[i * n + k0 + j] = (diag_blk && i - k0 == j) ? 1.0 : 0.0;
  }
}

// In-place inverse of the b x b block W (b <= NB = 128) by Gauss-Jordan with partial row
// pivoting, one workgroup of 1024 threads. Thread t holds column j = t % 128 of rows
// g + 8 k (g = t / 128, k = 0..15) in registers; LDS carries only what a step shares: the
// pivot candidates, the pivot row and the pivot column. Step p: the row r >= p of largest
// |W[r][p]| is exchanged with row p (perm[p] = r), then the usual in-place elimination with that
// pivot. Pivoting the rows yields (P W)^-1 = W^-1 P^T, so the column exchanges are undone in
// reverse order: column c of the result is the eliminated column src[c]. A zero or non-finite
// pivot sets *bad.
constexpr int GJ_RPT = NB / 8;  // rows per thread

// w[k] for a k known only at run time, selected without indexing the register array
__device__ __forceinline__ double gj_get(const double (&w)[GJ_RPT], int k) {
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < GJ_RPT; ++q) v = q == k ? w[q] : v;
  return v;
}
__device__ __forceinline__ void gj_set(double (&w)[GJ_RPT], int k, double v) {
#pragma unroll
  for (int q = 0; q < GJ_RPT; ++q) w[q] = q == k ? v : w[q];
}

__global__ __launch_bounds__(1024) void k_small_gj(double* W, int b, int* bad) {
  __shared__ double rowp[NB], colp[NB], rowr[NB];
  __shared__ double cv[8];
  __shared__ int ci[8];
  __shared__ int perm[NB], src[NB];
  __shared__ int piv_row;
  const int tid = threadIdx.x, j = tid & (NB - 1), g = tid >> 7;
  double w[GJ_RPT];
#pragma unroll
  for (int k = 0; k < GJ_RPT; ++k) {
    const int i = g + 8 * k;
    w[k] = (i < b && j < b) ? W[i * b + j] : 0.0;
  }
  for (int p = 0; p < b; ++p) {
    // pivot search in column p: the eight threads holding it reduce their rows >= p
    if (j == p) {
      double best = -1.0;
      int br = p;
#pragma unroll
      for (int k = 0; k < GJ_RPT; ++k) {
        const int i = g + 8 * k;
        const double v = fabs(w[k]);
        if (i >= p && i < b && v > best) {
          best = v;
          br = i;
        }
      }
      cv[g] = best;
      ci[g] = br;
    }
    __syncthreads();
    if (tid == 0) {
      double best = cv[0];
      int br = ci[0];
      for (int q = 1; q < 8; ++q)
        if (cv[q] > best || (cv[q] == best && ci[q] < br)) {
          best = cv[q];
          br = ci[q];
        }
      piv_row = br;
      perm[p] = br;
    }
    __syncthreads();
    const int r = piv_row;
    const int gp = p & 7, kp = p >> 3, gr = r & 7, kr = r >> 3;
    // rows p and r through LDS: row p's old values to rowp, row r's to rowr
    if (g == gp) rowp[j] = gj_get(w, kp);
    if (g == gr) rowr[j] = gj_get(w, kr);
    __syncthreads();
    if (r != p) {
      if (g == gp) gj_set(w, kp, rowr[j]);
      if (g == gr) gj_set(w, kr, rowp[j]);
    }
    __syncthreads();
    // the pivot row (after the exchange) and the pivot column
    if (g == gp) rowp[j] = gj_get(w, kp);
    if (j == p)
#pragma unroll
      for (int k = 0; k < GJ_RPT; ++k) colp[g + 8 * k] = w[k];
    __syncthreads();
    const double d = rowp[p];
    if (tid == 0 && (!(fabs(d) > 0.0) || !isfinite(d))) atomicOr(bad, 1);
    const double ip = 1.0 / d;
    const double rj = rowp[j];
#pragma unroll
    for (int k = 0; k < GJ_RPT; ++k) {
      const int i = g + 8 * k;
      const double ci_ = colp[i];
      double v;
      if (i == p && j == p) v = ip;
      else if (i == p) v = rj * ip;
      else if (j == p) v = -ci_ * ip;
      else v = w[k] - ci_ * rj * ip;
      w[k] = v;
    }
    __syncthreads();  // rowp, colp and the candidates are rewritten by the next step
  }
  // undo the row exchanges as column exchanges, last first: output column c = column src[c]
  if (tid == 0) {
    for (int c = 0; c < b; ++c) src[c] = c;
    for (int p = b - 1; p >= 0; --p) {
      const int r = perm[p];
      const int t = src[p];
      src[p] = src[r];
      src[r] = t;
    }
    for (int c = 0; c < b; ++c) perm[src[c]] = c;  // perm now maps a source column to its output
  }
  __syncthreads();
  if (j < b) {
    const int c = perm[j];
#pragma unroll
    for (int k = 0; k < GJ_RPT; ++k) {
      const int i = g + 8 * k;
      if (i < b) W[i * b + c] = w[k];
    }
  }
}

// Probe vectors for inverse_residual: X[r][i] = +-1 from an integer hash of (r, i).
__global__ void k_probe(double* X, int64_t n, int rows) {
  const int64_t total = n * rows;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    uint64_t h = (uint64_t)e * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    h ^= h >> 31;
    h *= 0xD6E8FEB86659FD93ull;
    h ^= h >> 32;
    X[e] = (h & 1) ? 1.0 : -1.0;
  }
}

// *out = max |Z| over `total` elements (one workgroup).
__global__ __launch_bounds__(1024) void k_maxabs(const double* Z, int64_t total, double* out) {
  __shared__ double m[1024];
  double v = 0.0;
  for (int64_t e = threadIdx.x; e < total; e += 1024) v = fmax(v, fabs(Z[e]));
  m[threadIdx.x] = v;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) m[threadIdx.x] = fmax(m[threadIdx.x], m[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (isfinite(m[0]) ? m[0] : INFINITY);
}

// Cholesky factorization of the b x b diagonal block at (k0, k0) of A in LDS (lower, right
// looking); writes L_KK back (zero above the diagonal) and its inverse W = L_KK^-1 (b x b, lower).
// A pivot that is not positive and finite sets *bad (the block is then garbage, never used).
__global__ __launch_bounds__(1024) void k_chol_block(double* A, int64_t n, int64_t k0, int b,
                                                    double* W, int* bad) {
  __shared__ double a[NB * NB];
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) a[e] = A[(k0 + e / b) * n + k0 + e % b];
  __syncthreads();
  for (int j = 0; j < b; ++j) {
    if (threadIdx.x == 0) {
      double d = a[j * b + j];
      if (!(d > 0.0) || !isfinite(d)) {
        atomicOr(bad, 1);
        d = 1.0;
      }
      a[j * b + j] = sqrt(d);
    }
    __syncthreads();
    const double p = a[j * b + j];
    for (int i = j + 1 + threadIdx.x; i < b; i += blockDim.x) a[i * b + j] /= p;
    __syncthreads();
    const int m = b - j - 1;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
      const int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k <= i) a[i * b + k] -= a[i * b + j] * a[k * b + j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
    const int i = e / b, k = e % b;
    A[(k0 + i) * n + k0 + k] = k <= i ? a[e] : 0.0;
  }
  // W = L^-1 by forward substitution, W[i][t] = -(sum_{t<=k<i} L[i][k] W[k][t]) / L[i][i] for
  // t < i and W[i][i] = 1 / L[i][i]: thread t owns column t of W (written and re-read by that
  // thread only), L comes from LDS.
  const int t = threadIdx.x;
  if (t < b) {
    for (int i = 0; i < b; ++i) {
      double v = 0.0;
      if (t < i) {
        double acc = 0.0;
        for (int k = t; k < i; ++k) acc += a[i * b + k] * W[k * b + t];
        v = -acc / a[i * b + i];
      } else if (t == i) {
        v = 1.0 / a[i * b + i];
      }
      W[i * b + t] = v;
    }
  }
}

// Zero the strict upper triangle of the n x n row-major A.
__global__ void k_zero_upper(double* A, int64_t n) {
  const int64_t nn = n * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nn; e += (int64_t)gridDim.x * 256)
    if (e % n > e / n) A[e] = 0.0;
}

__global__ void k_nonfinite(const double* A, int64_t n, int* bad) {
  int f = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    if (!isfinite(A[e])) f = 1;
  if (f) atomicOr(bad, 1);
}

}  // namespace

size_t invert_work_doubles(int64_t n) {
  // U (n x NB), R (NB x n), W (NB x NB), flag word
  return (size_t)n * NB * 2 + (size_t)NB * NB + 8;
}

hipError_t invert_in_place(double* A, int64_t n, double* work, hipStream_t s, int* bad_host) {
  double* U = work;
  double* R = U + (size_t)n * NB;
  double* W = R + (size_t)n * NB;
  int* flag = reinterpret_cast<int*>(W + (size_t)NB * NB);
  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), s);
  if (e != hipSuccess) return e;
  for (int64_t k0 = 0; k0 < n; k0 += NB) {
    const int b = (int)((n - k0) < NB ? (n - k0) : NB);
    int64_t total = n * b;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_panel, dim3(blocks), dim3(256), 0, s, A, n, k0, b, U, W);
    hipLaunchKernelGGL(k_small_gj, dim3(1), dim3(1024), 0, s, W, b, flag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // R = W * A[k0:k0+b, :]   (b x n, K = b)
    GemmDesc d{CF64, T_F64, T_F64, T_F64, T_F64, KC, RC, 1, 1};
    GemmOp op{};
    op.M = b; op.N = (int)n; op.nseg = 1;
    op.A[0] = W; op.lda[0] = b;
    op.B[0] = A + k0 * n; op.ldb[0] = n;
    op.K[0] = b;
    op.C = R; op.ldc = n;
    op.X = nullptr; op.ldx = 0;
    op.alpha = 1.0; op.beta = 0.0;
    if ((e = gemm_launch(d, &op, 1, nullptr, nullptr, 0, s)) != hipSuccess) return e;
    // A = A - U R   (n x n, K = b), in place; 128 x 128 tiles at two workgroups per CU (this
    // update streams the whole matrix once per pivot block: 0.27 against 0.36 s for the
    // 13000-orbital inverse with one workgroup per CU)
    GemmDesc d2{CF64, T_F64, T_F64, T_F64, T_F64, KC, RC, 4, 1};
    GemmOp op2{};
    op2.M = (int)n; op2.N = (int)n; op2.nseg = 1;
    op2.A[0] = U; op2.lda[0] = b;
    op2.B[0] = R; op2.ldb[0] = n;
    op2.K[0] = b;
    op2.C = A; op2.ldc = n;
    op2.X = A; op2.ldx = n;
    op2.alpha = -1.0; op2.beta = 1.0;
    if ((e = gemm_launch(d2, &op2, 1, nullptr, nullptr, 0, s)) != hipSuccess) return e;
  }
  const int64_t nn = n * n;
  int blocks = (int)((nn + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_nonfinite, dim3(blocks), dim3(256), 0, s, A, nn, flag);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int h = 0;
  if ((e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  *bad_host = h;
  return hipSuccess;
}

size_t inverse_residual_work_doubles(int64_t n) { return (size_t)3 * PROBES * n + 8; }

// max_ij |(X P A)_ij - X_ij| for PROBES rows X of +-1 entries, with A = S + (1/tau) T (T null:
// A = S): X P A = X exactly when P = A^-1, and the residual of a backward-stable inverse is
// ~ eps times the growth of the elimination. P, S, T are symmetric, so every product reads
// its operator k-contiguous.
hipError_t inverse_residual(const double* P, const double* S, const double* T, double inv_tau,
                            int64_t n, double* work, hipStream_t s, double* res_host) {
  double* X = work;
  double* Y = X + (size_t)PROBES * n;
  double* Z = Y + (size_t)PROBES * n;
  double* out = Z + (size_t)PROBES * n;
  const int64_t total = (int64_t)PROBES * n;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_probe, dim3(blocks), dim3(256), 0, s, X, n, PROBES);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  GemmDesc d{CF64, T_F64, T_F64, T_F64, T_F64, KC, KC, 0, 1};
  auto op_of = [&](const double* A, const double* B, double* C, const double* Xa, double alpha,
                   double beta) {
    GemmOp op{};
    op.M = PROBES; op.N = (int)n; op.nseg = 1;
    op.A[0] = A; op.lda[0] = n;
    op.B[0] = B; op.ldb[0] = n;
    op.K[0] = (int)n;
    op.C = C; op.ldc = n;
    op.X = Xa; op.ldx = Xa ? n : 0;
    op.alpha = alpha; op.beta = beta;
    return op;
  };
  GemmOp o1 = op_of(X, P, Y, nullptr, 1.0, 0.0);  // Y = X P
  if ((e = gemm_launch(d, &o1, 1, nullptr, nullptr, 0, s)) != hipSuccess) return e;
  GemmOp o2 = op_of(Y, S, Z, X, 1.0, -1.0);  // Z = Y S - X
  if ((e = gemm_launch(d, &o2, 1, nullptr, nullptr, 0, s)) != hipSuccess) return e;
  if (T) {
    GemmOp o3 = op_of(Y, T, Z, Z, inv_tau, 1.0);  // Z += (1/tau) Y T
    if ((e = gemm_launch(d, &o3, 1, nullptr, nullptr, 0, s)) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_maxabs, dim3(1), dim3(1024), 0, s, Z, total, out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(res_host, out, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return e;
  return hipStreamSynchronize(s);
}

size_t cholesky_work_doubles() { return (size_t)NB * NB + 8; }

// Blocked right-looking Cholesky S = L L^T in place on A (n x n, row-major, symmetric positive
// definite): for each block column K (width b <= 128), factor A_KK and invert its triangle in one
// workgroup (W), L_IK = A_IK W^T for the rows below (one 128-wide GEMM tile per row block, so
// the in-place update reads each row block before writing it), then A_II -= L_IK L_IK^T on the
// whole trailing square (GEMM). The strict upper triangle is zeroed at the end.
hipError_t cholesky_in_place(double* A, int64_t n, double* work, hipStream_t s, int* bad_host) {
  double* W = work;
  int* flag = reinterpret_cast<int*>(W + (size_t)NB * NB);
  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), s);
  if (e != hipSuccess) return e;
  for (int64_t k0 = 0; k0 < n; k0 += NB) {
    const int b = (int)((n - k0) < NB ? (n - k0) : NB);
    hipLaunchKernelGGL(k_chol_block, dim3(1), dim3(1024), 0, s, A, n, k0, b, W, flag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t r0 = k0 + b, R = n - r0;
    if (R <= 0) break;
    double* panel = A + r0 * n + k0;
    // L_IK = A_IK W^T: 128 x 128 tiles, one tile across the b columns (in place)
    GemmDesc d{CF64, T_F64, T_F64, T_F64, T_F64, KC, KC, 0, 1};
    GemmOp op{};
    op.M = (int)R; op.N = b; op.nseg = 1;
    op.A[0] = panel; op.lda[0] = n;
    op.B[0] = W; op.ldb[0] = b;
    op.K[0] = b;
    op.C = panel; op.ldc = n;
    op.alpha = 1.0; op.beta = 0.0;
    if ((e = gemm_launch(d, &op, 1, nullptr, nullptr, 0, s)) != hipSuccess) return e;
    // A_II -= L_IK L_IK^T (trailing square, in place)
    GemmOp op2{};
    op2.M = (int)R; op2.N = (int)R; op2.nseg = 1;
    op2.A[0] = panel; op2.lda[0] = n;
    op2.B[0] = panel; op2.ldb[0] = n;
    op2.K[0] = b;
    op2.C = A + r0 * n + r0; op2.ldc = n;
    op2.X = A + r0 * n + r0; op2.ldx = n;
    op2.alpha = -1.0; op2.beta = 1.0;
    if ((e = gemm_launch(d, &op2, 1, nullptr, nullptr, 0, s)) != hipSuccess) return e;
  }
  const int64_t nn = n * n;
  int blocks = (int)((nn + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_zero_upper, dim3(blocks), dim3(256), 0, s, A, n);
  hipLaunchKernelGGL(k_nonfinite, dim3(blocks), dim3(256), 0, s, A, nn, flag);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int h = 0;
  if ((e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  *bad_host = h;
  return hipSuccess;
}

}  // namespace omm
