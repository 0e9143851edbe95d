// GEMM launcher: picks the instantiation for a descriptor, sizes the grid (XCD-remapped tile
// ids, split-K along y, up to 4 same-shape products along z) and reduces split-K partials in a
// fixed order.
#include "omm_gemm_impl.h"

namespace omm {
namespace gemm_detail {
gemm_fn pick_f64(const GemmDesc& d);
gemm_fn pick_f32(const GemmDesc& d);
gemm_fn pick_bf16x3(const GemmDesc& d);
gemm_fn pick_bf16x2(const GemmDesc& d);
sk_fn pick_sk_bf16x3(const GemmDesc& d);
sk_fn pick_sk_bf16x2(const GemmDesc& d);
grouped_fn pick_grouped_f32(const GemmDesc& d);
grouped_fn pick_grouped_f64(const GemmDesc& d);

namespace {
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
    const int row = (int)(idx / op.N), col = (int)(idx % op.N);
    if (op.tri && row > col) continue;  // mirrored afterwards (its tile may not have run)
    for (int sp = 0; sp < nsplit; ++sp) s += ws[((int64_t)sp * nops + blockIdx.y) * mn + idx];
    double v = op.alpha * s;
    if (op.X) v += op.beta * (double)ldg<TX>(op.X, (int64_t)row * op.ldx + col);
    store_out<TC>(op, row, col, v);
  }
}
// C[i][j] = C[j][i] for i > j of every symmetric (tri) product: 32 x 32 blocks on and below the
// diagonal, each read transposed through LDS from its mirror block.
template <typename TC>
__global__ __launch_bounds__(256) void mirror_lower(GemmBatch batch, const int* done) {
  if (done && *done) return;
  const GemmOp& op = batch.op[blockIdx.z];
  if (!op.tri) return;
  const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;  // destination block (rows bi, cols bj)
  if (bj > bi || bi >= op.M) return;
  __shared__ TC t[32][33];
  TC* C = static_cast<TC*>(op.C);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {  // source block: rows bj, cols bi
    const int i = bj + r, j = bi + tx;
    if (i < op.M && j < op.N) t[r][tx] = C[(int64_t)i * op.ldc + j];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = bi + r, j = bj + tx;
    if (i < op.M && j < op.N && i > j) C[(int64_t)i * op.ldc + j] = t[tx][r];
  }
}
}  // namespace
}  // namespace gemm_detail

using namespace gemm_detail;

size_t gemm_splitk_ws_bytes(const GemmOp* ops, int nops, int splitk) {
  if (splitk <= 1) return 0;
  return (size_t)splitk * nops * (size_t)ops[0].M * ops[0].N * sizeof(double);
}

size_t gemm_ws_bytes(const GemmDesc& d, const GemmOp* ops, int nops) {
  if (d.tile == 6) return (size_t)2 * SK_GRID * DMA_BM * DMA_BN * sizeof(float);
  return gemm_splitk_ws_bytes(ops, nops, d.splitk);
}

int gemm_num_tiles() { return NTILES; }
int gemm_grouped_num_tiles() { return NTILES_GROUPED; }

namespace {
// Preconditions of the direct-to-LDS tile: 16-byte aligned planes, leading dimensions that are
// multiples of 8, and K-segment boundaries on 8-element boundaries.
bool dma_ok(const GemmDesc& d, const GemmOp* ops, int nops) {
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  for (int i = 0; i < nops; ++i) {
    const GemmOp& op = ops[i];
    if (op.nseg == 2 && op.K[0] % 8 != 0) return false;
    for (int g = 0; g < op.nseg; ++g) {
      if (op.lda[g] % 8 != 0 || op.ldb[g] % 8 != 0) return false;
      // lane addresses are 32-bit byte offsets from the plane base
      constexpr int64_t lim = (int64_t)1 << 31;
      if ((int64_t)op.M * op.lda[g] >= lim || (int64_t)op.N * op.ldb[g] >= lim) return false;
      if (!al(op.A[g]) || !al(op.B[g])) return false;
      if (!one_plane_a(d.compute) && !al(op.Alo[g])) return false;
      if (!one_plane_b(d.compute) && !al(op.Blo[g])) return false;
    }
  }
  return true;
}
}  // namespace

namespace {
sk_fn pick_sk(const GemmDesc& d) {
  if (d.compute == CBF16X3) return pick_sk_bf16x3(d);
  if (d.compute == CBF16X2A || d.compute == CBF16X2B || d.compute == CBF16X1)
    return pick_sk_bf16x2(d);
  return nullptr;
}
}  // namespace

bool gemm_supported(const GemmDesc& d) {
  if (d.tile < 0 || d.tile >= NTILES) return false;
  if (d.tile == 6) return d.splitk <= 1 && pick_sk(d) != nullptr;
  if (d.tile == 7 && d.splitk > 1) return false;
  if (d.compute == CF64) return pick_f64(d) != nullptr;
  if (d.compute == CF32) return pick_f32(d) != nullptr;
  if (d.compute == CBF16X3) return pick_bf16x3(d) != nullptr;
  if (d.compute == CBF16X2A || d.compute == CBF16X2B || d.compute == CBF16X1)
    return pick_bf16x2(d) != nullptr;
  return false;
}

hipError_t gemm_grouped_launch(const GemmDesc& d, const GemmOp* d_ops, const int* d_tile_start,
                               const int* const* d_done, int nops, int grid, hipStream_t s) {
  if ((d.compute != CF32 && d.compute != CF64) || nops < 1 || grid < 1)
    return hipErrorInvalidValue;
  grouped_fn fn = d.compute == CF64 ? pick_grouped_f64(d) : pick_grouped_f32(d);
  if (!fn) return hipErrorInvalidValue;
  GroupedArgs g{d_ops, d_tile_start, d_done, nops};
  hipLaunchKernelGGL(fn, dim3(grid), dim3(tile_threads(d.tile, d.compute)), 0, s, g);
  return hipGetLastError();
}

int gemm_tile_rows(int tile, int mode) { return tile_bm(tile, mode); }
int gemm_tile_cols(int tile, int mode) { return tile_bn(tile, mode); }

namespace {
hipError_t launch_products(const GemmDesc& d, const GemmOp* ops, int nops, const int* done,
                           double* ws, size_t ws_bytes, hipStream_t s) {
  if (nops < 1 || nops > 4) return hipErrorInvalidValue;
  GemmBatch b;
  for (int i = 0; i < nops; ++i) {
    b.op[i] = ops[i];
    if (ops[i].M != ops[0].M || ops[i].N != ops[0].N) return hipErrorInvalidValue;
    if (ops[i].nseg < 1 || ops[i].nseg > 2) return hipErrorInvalidValue;
  }
  const int M = ops[0].M, N = ops[0].N;
  if (M <= 0 || N <= 0) return hipSuccess;
  if (d.tile < 0 || d.tile >= NTILES) return hipErrorInvalidValue;
  GemmDesc dd = d;
  bool sparse = false;
  for (int i = 0; i < nops; ++i) sparse |= ops[i].kptr != nullptr;
  if (sparse) {
    // block-sparse B lists are read over the whole K range: BF16 modes by the direct-to-LDS
    // tile (which stages a column tile's list in LDS), FP64/FP32 by the register tiles (whose
    // column tiles, 64 to 256 wide, lie within one 256-column list tile)
    for (int i = 0; i < nops; ++i)
      if (ops[i].nseg != 1 || !ops[i].kidx) return hipErrorInvalidValue;
    if (is_bf16_mode(dd.compute)) {
      for (int i = 0; i < nops; ++i)
        if ((ops[i].K[0] + SPARSE_BK - 1) / SPARSE_BK > SPARSE_KL_MAX) return hipErrorInvalidValue;
      if (!dma_ok(dd, ops, nops)) return hipErrorInvalidValue;
      dd.tile = 5;
    } else if (dd.tile > 4) {
      return hipErrorInvalidValue;
    }
    dd.splitk = 1;
  }
  if (dd.tile == 6) {
    if (dma_ok(dd, ops, nops)) {
      sk_fn fn = pick_sk(dd);
      if (!fn || dd.splitk > 1) return hipErrorInvalidValue;
      if (!ws || ws_bytes < gemm_ws_bytes(dd, ops, nops)) return hipErrorInvalidValue;
      int tiles = 0;  // tile-ops over all products
      for (int i = 0; i < nops; ++i) tiles += op_tiles(ops[i], DMA_BM, DMA_BN);
      const int ktot = ops[0].K[0] + (ops[0].nseg > 1 ? ops[0].K[1] : 0);
      for (int i = 1; i < nops; ++i)
        if (ops[i].nseg != ops[0].nseg || ops[i].K[0] != ops[0].K[0] ||
            (ops[0].nseg > 1 && ops[i].K[1] != ops[0].K[1]))
          return hipErrorInvalidValue;  // one K schedule for every product of the launch
      SkArgs a;
      a.T = tiles;
      a.nops = nops;
      a.nk = (ktot + DMA_BK - 1) / DMA_BK;
      a.R = a.T / SK_GRID;
      a.W = (int64_t)(a.T - a.R * SK_GRID) * a.nk;
      float* parts = reinterpret_cast<float*>(ws);
      hipLaunchKernelGGL(fn, dim3(SK_GRID), dim3(512), 0, s, b, done, a, parts);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess || a.W == 0) return e;
      sk_fixup_fn fx = dd.tc == T_F64   ? gemm_sk_fixup<double, double>
                       : dd.tx == T_F64 ? gemm_sk_fixup<float, double>
                                        : gemm_sk_fixup<float, float>;
      if (dd.tc == T_F64 && dd.tx != T_F64) return hipErrorInvalidValue;
      hipLaunchKernelGGL(fx, dim3(a.T - a.R * SK_GRID, SK_FIX_CHUNKS), dim3(256), 0, s, b, done, a,
                         SK_GRID, (const float*)parts);
      return hipGetLastError();
    }
    dd.tile = 4;  // same 256 x 256 tile on the register path, one workgroup per tile
    dd.splitk = 1;
  }
  if (dd.tile == 5 && !dma_ok(dd, ops, nops)) dd.tile = 4;  // same 256 x 256 tile, register path
  gemm_fn fn = nullptr;
  if (dd.compute == CF64) fn = pick_f64(dd);
  else if (dd.compute == CF32) fn = pick_f32(dd);
  else if (dd.compute == CBF16X3) fn = pick_bf16x3(dd);
  else if (dd.compute == CBF16X2A || dd.compute == CBF16X2B || dd.compute == CBF16X1)
    fn = pick_bf16x2(dd);
  if (!fn) return hipErrorInvalidValue;
  const int bm = tile_bm(dd.tile, dd.compute), bn = tile_bn(dd.tile, dd.compute);
  const int tiles = ((M + bm - 1) / bm) * ((N + bn - 1) / bn);
  const int per = (tiles + 7) / 8;
  const int splitk = dd.splitk > 1 ? dd.splitk : 1;
  if (splitk > 1 && (!ws || ws_bytes < gemm_splitk_ws_bytes(ops, nops, splitk)))
    return hipErrorInvalidValue;
  dim3 grid(8 * per, splitk, nops);
  hipLaunchKernelGGL(fn, grid, dim3(tile_threads(dd.tile, dd.compute)), 0, s, b, done, splitk, ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splitk == 1) return e;
  const int64_t mn = (int64_t)M * N;
  int blocks = (int)((mn + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  dim3 rgrid(blocks, nops);
  void (*red)(GemmBatch, const int*, int, const double*) = nullptr;
  if (dd.tc == T_F64) red = dd.tx == T_F64 ? splitk_reduce<double, double> : splitk_reduce<double, float>;
  else red = dd.tx == T_F64 ? splitk_reduce<float, double> : splitk_reduce<float, float>;
  hipLaunchKernelGGL(red, rgrid, dim3(256), 0, s, b, done, splitk, (const double*)ws);
  return hipGetLastError();
}
}  // namespace

hipError_t gemm_launch(const GemmDesc& d, const GemmOp* ops, int nops, const int* done, double* ws,
                       size_t ws_bytes, hipStream_t s) {
  if (nops < 1 || nops > 4) return hipErrorInvalidValue;
  bool tri = false;
  for (int i = 0; i < nops; ++i) {
    if (!ops[i].tri) continue;
    if (ops[i].M != ops[i].N || ops[i].Chi || ops[i].kptr) return hipErrorInvalidValue;
    tri = true;
  }
  hipError_t e = launch_products(d, ops, nops, done, ws, ws_bytes, s);
  // the one-wave tile writes both halves of a symmetric result itself
  if (e != hipSuccess || !tri || ops[0].M <= 0 || d.tile == 7) return e;
  GemmBatch b;
  for (int i = 0; i < nops; ++i) b.op[i] = ops[i];
  const int nb = (ops[0].M + 31) / 32;
  if (d.tc == T_F64)
    hipLaunchKernelGGL(mirror_lower<double>, dim3(nb, nb, nops), dim3(256), 0, s, b, done);
  else
    hipLaunchKernelGGL(mirror_lower<float>, dim3(nb, nb, nops), dim3(256), 0, s, b, done);
  return hipGetLastError();
}

}  // namespace omm
