// One-time FP64 inversion for the preconditioner P = (S + T/tau)^-1 (Sec. 2.4, Eq. 17): an
// in-place blocked Gauss-Jordan sweep. The paper inverts once per MD step with a library
// LU; here each block column costs one tiny pivot-block inversion plus two MFMA GEMMs, so the
// 2 n^3 flops run on matrix cores.
//
// Step for pivot block K (width b), with A the current matrix:
//   U  = A[:, K] with its diagonal block replaced by A_KK - I      (column panel copy)
//   W  = A_KK^-1                                                    (one workgroup)
//   A[:, K] = e_K  (zero column panel, identity diagonal block)
//   R  = W A[K, :]                                                  (b x n GEMM)
//   A -= U R                                                        (rank-b GEMM update)
// which leaves A[K,K] = W, A[K,J] = W A_KJ, A[I,K] = -A_IK W and the Schur update elsewhere;
// after the last block A holds the inverse. No pivoting: S + T/tau is symmetric positive
// definite for the workloads here. A zero or non-finite pivot is reported, never hidden.
#include <math.h>

#include "omm_internal.h"

namespace omm {
namespace {

constexpr int NB = 128;

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

// In-place Gauss-Jordan inverse of the b x b block W by one workgroup.
__global__ __launch_bounds__(1024) void k_small_gj(double* W, int b, int* bad) {
  __shared__ double rowp[NB], colp[NB];
  __shared__ double piv;
  for (int p = 0; p < b; ++p) {
    if (threadIdx.x == 0) {
      const double d = W[p * b + p];
      if (!(fabs(d) > 0.0) || !isfinite(d)) atomicOr(bad, 1);
      piv = 1.0 / d;
    }
    for (int t = threadIdx.x; t < b; t += blockDim.x) {
      rowp[t] = W[p * b + t];
      colp[t] = W[t * b + p];
    }
    __syncthreads();
    const double ip = piv;
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
      const int i = e / b, j = e % b;
      double v;
      if (i == p && j == p) v = ip;
      else if (i == p) v = rowp[j] * ip;
      else if (j == p) v = -colp[i] * ip;
      else v = W[e] - colp[i] * rowp[j] * ip;
      W[e] = v;
    }
    __syncthreads();
  }
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
    // A = A - U R   (n x n, K = b), in place
    GemmDesc d2{CF64, T_F64, T_F64, T_F64, T_F64, KC, RC, 0, 1};
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
