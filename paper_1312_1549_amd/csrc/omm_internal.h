// Internal declarations shared by the translation units of libomm (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace omm {

// Device-resident scalars of one minimization. Every iteration kernel reads `done` first and
// returns at once when it is non-zero, so iterations launched after convergence cost nothing.
struct DevState {
  double E;          // functional at the current C
  double E_prev;     // functional before the last line search
  double x;          // last line-search step
  double beta;       // last Polak-Ribiere coefficient
  double pg_g;       // <PG, G> of the current gradient (denominator of the next beta)
  double alpha[5];   // last quartic coefficients
  double rel_change; // |2 (E - E_prev)| / |E + E_prev|
  double tol;
  int iter;          // completed line searches
  int max_iter;
  int done;          // 0 running, 1 converged, 2 max_iter, <0 error code
  int pad;
};

// Operand layout of a GEMM operand X with outer index r (row of A, column of B) and inner k:
//   KC: element (r, k) at X[r * ld + k]   (k contiguous)
//   RC: element (r, k) at X[k * ld + r]   (r contiguous)
enum Layout : int { KC = 0, RC = 1 };

// CBF16X3: both operands are hi/lo bf16 plane pairs, three products per K step (lo*hi, hi*lo,
// hi*hi). CBF16X2A / CBF16X2B: A (B) holds exact bf16 values in its hi plane alone, so two
// products (hi*lo + hi*hi) carry the same accuracy. CBF16X1: both operands are single planes of
// exact bf16 values, one product (the product of the two bf16 matrices, FP32 sums).
enum Compute : int { CF64 = 0, CF32 = 1, CBF16X3 = 2, CBF16X2A = 3, CBF16X2B = 4, CBF16X1 = 5 };
constexpr bool is_bf16_mode(int m) { return m >= CBF16X3; }
constexpr bool one_plane_a(int m) { return m == CBF16X2A || m == CBF16X1; }
constexpr bool one_plane_b(int m) { return m == CBF16X2B || m == CBF16X1; }

// T_BF16P: a pair of bf16 planes (hi, lo) with a = hi + lo, pointers in A/Alo (B/Blo).
enum ElemType : int { T_F64 = 0, T_F32 = 1, T_BF16P = 2 };

struct GemmOp {
  int M, N;            // output rows, columns
  int nseg;            // 1 or 2 summed K segments
  const void* A[2];
  const void* B[2];
  const void* Alo[2];  // lo planes (T_BF16P operands only)
  const void* Blo[2];
  int64_t lda[2], ldb[2];
  int K[2];
  void* C;             // output
  int64_t ldc;
  const void* X;       // epilogue addend (may alias C), nullable
  int64_t ldx;
  double alpha, beta;  // C = alpha * sum_seg A_seg B_seg + beta * X
  // Block-sparse B (one segment, direct-to-LDS tile only; nullable = dense): for column tile t
  // of the 256-wide output tiling, kidx[kptr[t] .. kptr[t + 1]) are the ascending 32-deep K
  // blocks in which that tile's rows of B are not all zero. The skipped blocks contribute exact
  // zeros, so the result equals the dense product (up to the sign of zero).
  const int* kptr;
  const int* kidx;
  // Optional bf16 planes of the output (nullable; row length ldp): Chi = bf16(c),
  // Clo = bf16(c - Chi) of each stored element c, for the next product's operand.
  void* Chi;
  void* Clo;
  int64_t ldp;
  // Symmetric result (M == N, no planes): only the tiles on and above the diagonal are computed
  // and the launcher then copies C[j][i] into C[i][j] for every i > j.
  int tri;
};

struct GemmDesc {
  int compute;         // Compute
  int ta, tb, tc, tx;  // ElemType of A, B, C, X
  int la, lb;          // Layout of A, B
  int tile;            // macro tile, see gemm_tile_rows / gemm_tile_cols (0..6)
  int splitk;          // >1: K split across workgroups, partials reduced in FP64 (needs ws)
};

// Launch up to 4 GEMMs that share a descriptor (one launch; blockIdx.z selects the op).
// `done` (nullable) makes the launch a no-op when *done != 0. `ws` is FP64 scratch for split-K.
hipError_t gemm_launch(const GemmDesc& d, const GemmOp* ops, int nops, const int* done,
                       double* ws, size_t ws_bytes, hipStream_t s);
size_t gemm_splitk_ws_bytes(const GemmOp* ops, int nops, int splitk);
// Workspace a launch with descriptor d needs (split-K partials, or stream-K tile parts).
size_t gemm_ws_bytes(const GemmDesc& d, const GemmOp* ops, int nops);
// Block pattern of the block-sparse B lists: 256-wide column tiles of the direct-to-LDS GEMM,
// 32-deep K blocks.
constexpr int SPARSE_BN = 256, SPARSE_BK = 32;
// Longest K-block list of one column tile (K up to 65536): the GEMM stages a tile's list in LDS.
constexpr int SPARSE_KL_MAX = 2048;
// flags[t * nkb + kb] = 1 iff some B[r][k] != 0 with r in column tile t and k in K block kb
// (B is n x n row-major; nkb = ceil(n / SPARSE_BK)).
hipError_t block_pattern(const double* B, int64_t n, unsigned char* flags, hipStream_t s);
// Exact real embedding of complex Hermitian problems (host side): the operator X = re + i im
// (n x n) becomes [[re, im], [-im, re]] (2n x 2n, acting on rows [Re c, Im c]); the complex
// m x n row matrix C becomes the 2m x 2n rows [Re c_i, Im c_i] and [-Im c_i, Re c_i].
void embed_operator(const double* re, const double* im, int64_t n, std::vector<double>& out);
void embed_rows(const double* re, const double* im, int64_t m, int64_t n, std::vector<double>& out);
int gemm_num_tiles();
int gemm_grouped_num_tiles();
bool gemm_supported(const GemmDesc& d);
int gemm_tile_rows(int tile, int mode);
int gemm_tile_cols(int tile, int mode);
// Grouped FP32 or FP64 products of uneven shapes in one persistent launch of `grid` workgroups.
// All arrays are device memory: nops ops, tile prefix sums (nops + 1, computed with the tile
// shape of d.tile), per-op done flags (entries nullable). No split-K.
hipError_t gemm_grouped_launch(const GemmDesc& d, const GemmOp* d_ops, const int* d_tile_start,
                               const int* const* d_done, int nops, int grid, hipStream_t s);

// ---- elementwise / reduction kernels (omm_kernels.hip) ----
// Number of per-block partial sums each reduction writes is at most RED_BLOCKS.
constexpr int RED_BLOCKS = 1024;
constexpr int NCOEF = 13;

hipError_t shift_hamiltonian(const double* H, const double* S, double eta, double* Hs, int64_t n,
                             hipStream_t s);
hipError_t convert_f64_f32(const double* src, float* dst, int64_t n, hipStream_t s);
// hi = bf16(x), lo = bf16(x - hi) (round to nearest even), skipped when st->done. src is rows x
// cols (contiguous); hi/lo rows have length ld (>= cols, a multiple of 4).
hipError_t split_bf16(const float* src, unsigned short* hi, unsigned short* lo, int64_t rows,
                      int64_t cols, int64_t ld, const DevState* st, hipStream_t s);
hipError_t split_bf16(const double* src, unsigned short* hi, unsigned short* lo, int64_t rows,
                      int64_t cols, int64_t ld, const DevState* st, hipStream_t s);
// Planes of the transpose: src is rows x cols row-major, hi/lo are cols x rows with row length
// ld >= rows.
hipError_t split_bf16_t(const float* src, unsigned short* hi, unsigned short* lo, int rows,
                        int cols, int64_t ld, const DevState* st, hipStream_t s);
hipError_t split_bf16_t(const double* src, unsigned short* hi, unsigned short* lo, int rows,
                        int cols, int64_t ld, const DevState* st, hipStream_t s);
// Real embedding of a complex matrix with 2 rh rows and 2 h columns (row length ld): rows
// rh .. 2 rh - 1 := [-X[r][h:2h], X[r][0:h]] of rows 0 .. rh - 1 (FP64 if f64, else FP32), and
// the same for the optional bf16 planes hi/lo (row length ldp). Skipped when st->done.
hipError_t pair_rows(void* X, bool f64, int64_t ld, unsigned short* hi, unsigned short* lo,
                     int64_t ldp, int rh, int h, const DevState* st, hipStream_t s);
hipError_t convert_f32_f64(const float* src, double* dst, int64_t n, hipStream_t s);
hipError_t copy_f64(const double* src, double* dst, int64_t n, hipStream_t s);
// dst = src, setting *diff to 1 when any element's bits change (*diff is not cleared)
hipError_t copy_compare_f64(const double* src, double* dst, int64_t n, int* diff, hipStream_t s);
hipError_t validate_symmetric(const double* A, int64_t n, double rtol, int* flags, hipStream_t s);
hipError_t symmetrize(double* A, int64_t n, hipStream_t s);

// Energy of (HW, SW): writes partials then finalizes into st (init = 1: first energy of a run).
hipError_t energy_init(const double* HW, const double* SW, int M, double* partials, DevState* st,
                       double* trace, hipStream_t s);

// Polak-Ribiere beta and D = -PG + beta D. With `hi` non-null D is rounded to bf16 and its bits
// are written to `hi` (the single-plane operand of the two-product GEMMs; rows of length ld,
// n / cols of them); the previous direction is then read back from `hi`, and D, which may be
// null, only receives a copy of the rounded values.
template <typename T, typename TP = T, typename TG = T>
hipError_t beta_and_direction(const TG* G, const TP* PG, const TG* Gprev, T* D, int64_t n, int first,
                              double* partials, DevState* st, hipStream_t s,
                              unsigned short* hi = nullptr, int64_t cols = 0, int64_t ld = 0);

hipError_t line_search(const double* HW, const double* SW, const double* H1, const double* S1,
                       const double* H2, const double* S2, int M, double* partials, DevState* st,
                       hipStream_t s);

// HD, SD (type TD) may be held in a narrower type than the state (FP32 products of the BF16
// scheme with an FP64 state).
template <typename T, typename TD = T>
hipError_t update_coefficients(T* C, const T* D, T* HC, const TD* HD, T* SC, const TD* SD,
                               int64_t n, const DevState* st, hipStream_t s);

// bf16 hi/lo planes of HC and SC (rows x cols, row length ld) and of their transposes (cols x
// rows, row length ldt).
struct StatePlanes {
  unsigned short *hc_hi, *hc_lo, *sc_hi, *sc_lo;
  unsigned short *hct_hi, *hct_lo, *sct_hi, *sct_lo;
  int64_t ld, ldt;
};
// update_coefficients (rows x cols arrays) fused with the splits of the new HC and SC into `p`
// (the same values split_bf16 and split_bf16_t would write). The direction is read from its bf16
// plane Dh (rows of length ldd; D is exact in bf16 in this scheme); SD null means SD = D (the
// reduced problem, S~ = I).
template <typename T, typename TD = T>
hipError_t update_coefficients_split(T* C, const unsigned short* Dh, int64_t ldd, T* HC,
                                     const TD* HD, T* SC, const TD* SD, int rows, int cols,
                                     const StatePlanes& p, const DevState* st, hipStream_t s);

hipError_t update_subspace(double* HW, double* SW, const double* H1, const double* S1,
                           const double* H2, const double* S2, int M, double* partials,
                           DevState* st, double* trace, hipStream_t s);

hipError_t identity_minus(const double* SW, double* out, int M, double diag, double scale,
                          hipStream_t s);
hipError_t axpby_f64(const double* a, const double* b, double* out, double ca, double cb, int64_t n,
                     hipStream_t s);
hipError_t scale_f64(double* a, double c, int64_t n, hipStream_t s);

// ---- grouped (batched) stages: one launch over many systems, blockIdx.y = system ----
struct SysDev {
  void *C, *HC, *SC, *G0, *G1, *PG, *D, *HD, *SD;  // M x N, FP32 (f64 = 0) or FP64 (f64 = 1)
  double *HW, *SW, *H1, *S1, *H2, *S2;             // M x M (FP64)
  double* partials;                                // GROUP_BLOCKS x NCOEF
  DevState* st;
  double* trace;                                   // max_iter + 2 entries
  int M, N;
  int precon;                                      // PG holds G P (else PG aliases G)
  int paired;  // real embedding of a complex system: products computed for the first M / 2 rows
  int f64;     // type of the M x N arrays
};
constexpr int GROUP_BLOCKS = 64;

hipError_t group_energy_init(const SysDev* d_sys, int nsys, hipStream_t s);
hipError_t group_direction(const SysDev* d_sys, int nsys, int parity, int first, hipStream_t s);
hipError_t group_line_search(const SysDev* d_sys, int nsys, hipStream_t s);
hipError_t group_update(const SysDev* d_sys, int nsys, hipStream_t s);
// Rows M/2 .. M-1 of the paired systems' products from rows 0 .. M/2-1 by the pair rotation
// (see pair_rows): which = 0 HC, SC; 1 HW, SW; 2 G of `parity`; 3 PG; 4 HD, SD; 5 H', S', H'',
// S''. max_m, max_n bound the systems' sizes (grid shape); stopped systems are skipped when
// check_done.
hipError_t group_pair_rows(const SysDev* d_sys, int nsys, int which, int parity, bool check_done,
                           int max_m, int max_n, hipStream_t s);

// ---- preconditioner (omm_precon.hip) ----
// In-place inverse of an n x n matrix by a blocked Gauss-Jordan sweep. Returns hipSuccess and
// sets *bad (host) to 1 if a pivot block was singular or a non-finite value appeared.
hipError_t invert_in_place(double* A, int64_t n, double* work, hipStream_t s, int* bad);
size_t invert_work_doubles(int64_t n);
// max_ij |(X P A - X)_ij| over 16 probe rows X of +-1 entries, A = S + inv_tau T (T nullable:
// A = S), written to *res (host) after a stream synchronization. P, S, T symmetric, n x n.
hipError_t inverse_residual(const double* P, const double* S, const double* T, double inv_tau,
                            int64_t n, double* work, hipStream_t s, double* res);
size_t inverse_residual_work_doubles(int64_t n);
// An inverse whose probe residual exceeds this is rejected (OMM_E_PRECON).
constexpr double INVERSE_RESIDUAL_LIMIT = 1e-8;
// Cholesky factorization S = L L^T in place (L lower, strict upper set to zero); *bad != 0 when
// a pivot is not positive (S not positive definite) or the result is not finite.
hipError_t cholesky_in_place(double* A, int64_t n, double* work, hipStream_t s, int* bad);
size_t cholesky_work_doubles();

}  // namespace omm
