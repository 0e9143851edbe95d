// Batched entry points: many independent (H, S) systems of uneven size in one set of launches.
//
// Every CG stage is one launch over all systems. The products are grouped persistent GEMMs that
// walk the concatenated tile lists of all systems (FP32 or FP64 MFMA, a system that has stopped
// is skipped through its device flag); the reductions, the line minimum and the updates are
// grouped kernels with one y-slice per system (FP64 accumulation). The first line search of a
// phase runs eagerly and autotunes the macro tile of each grouped product; then two line
// searches are captured in a hipGraph and the graph is replayed until every system has
// stopped. Setup (shift, preconditioner inverse, FP32 copies) is per system.
//
// Precision: an FP32 phase (FP32 products and state), an FP64 phase, or the FP32 phase to the
// looser tolerance omm_batch_set_mixed_tol() followed by an FP64 phase from its C to `tol`
// (the refinement of the single-system OMM_FP32 mode, here in grouped launches as well).
#include <algorithm>
#include <math.h>

#include <string>
#include <vector>

#include "../../include/omm.h"
#include "omm_internal.h"

using namespace omm;

namespace {

struct BSys {
  int64_t N = 0, M = 0;
  double *H = nullptr, *S = nullptr, *T = nullptr;  // FP64 inputs
  bool have_T = false, have_HS = false;
  double *Hs64 = nullptr, *P64 = nullptr, *C64 = nullptr;
  // FP64 phase: M x N state and products (C64 is its C)
  double *HC64 = nullptr, *SC64 = nullptr, *G0_64 = nullptr, *G1_64 = nullptr, *PG64 = nullptr,
         *D64 = nullptr, *HD64 = nullptr, *SD64 = nullptr;
  bool c64_current = false;  // the latest C is C64 (an FP64 phase ran last)
  float *Hs = nullptr, *S32 = nullptr, *P = nullptr;
  float *C = nullptr, *HC = nullptr, *SC = nullptr, *G0 = nullptr, *G1 = nullptr, *PG = nullptr,
        *D = nullptr, *HD = nullptr, *SD = nullptr;
  double *HW = nullptr, *SW = nullptr, *H1 = nullptr, *S1 = nullptr, *H2 = nullptr, *S2 = nullptr;
  double* partials = nullptr;
  double* trace = nullptr;
  int trace_cap = 0;
  int p_kind = -1;  // -1 not built, 0 none, 1 S^-1, 2 (S + T/tau)^-1
  double p_tau = 0.0;
  bool p32_valid = false;  // P holds the FP32 copy of P64
  bool have_C = false;
};

// One grouped product: host op list, device copies, chosen macro tile.
struct OpList {
  GemmDesc d{};
  std::vector<GemmOp> ops;
  std::vector<const int*> done;
  GemmOp* d_ops = nullptr;
  int* d_tiles = nullptr;
  const int** d_done = nullptr;
  int cap = 0;
  int grid = 0;
  bool tuned = false;
};

}  // namespace

// The grouped products of one phase's CG stages.
struct PhaseLists {
  OpList init1, init2, grad[2], pg[2], hdsd, proj;
  std::vector<OpList*> all() {
    return {&init1, &init2, &grad[0], &grad[1], &pg[0], &pg[1], &hdsd, &proj};
  }
};

struct omm_batch {
  std::vector<BSys> sys;
  hipStream_t stream = nullptr;
  DevState* st = nullptr;       // nsys, device
  DevState* st_host = nullptr;  // nsys, pinned
  SysDev* d_sys = nullptr;      // FP32 phase
  SysDev* d_sys64 = nullptr;    // FP64 phase
  double* inv_work = nullptr;
  size_t inv_cap = 0;
  int* d_cmp = nullptr;  // change flag of omm_batch_set_HS's S / T comparison, then the two
                         // flags (non-finite, asymmetric) of the device-input validation
  PhaseLists L32, L64;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int mode = OMM_FP32;  // OMM_FP32 or OMM_FP64
  bool refine = false;  // OMM_FP32: FP64 phase after the FP32 one
  double mixed_tol = 1e-9;
  std::vector<int> iters, iters32, iters64;
  std::vector<double> E;
  std::string err;
  // complex Hermitian systems (k-points) held as their real embeddings (sizes 2N, 2M)
  bool cplx = false;
  std::vector<int64_t> Nc, Mc;
};

namespace {

int bfail(omm_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  return code;
}

#define BHIP(b, x)                                                                     \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) return bfail(b, OMM_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define BTRY(x)                  \
  do {                           \
    int r_ = (x);                \
    if (r_ != OMM_OK) return r_; \
  } while (0)

template <typename P>
int balloc(omm_batch* b, P** p, size_t n) {
  if (*p) return OMM_OK;
  if (hipMalloc((void**)p, (n ? n : 1) * sizeof(P)) != hipSuccess) {
    *p = nullptr;
    return bfail(b, OMM_E_ALLOC, "hipMalloc failed");
  }
  return OMM_OK;
}

template <typename P>
void bfree(P*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void free_list(OpList& L) {
  bfree(L.d_ops);
  bfree(L.d_tiles);
  if (L.d_done) (void)hipFree((void*)L.d_done);
  L.d_done = nullptr;
  L.cap = 0;
}

void free_sys(BSys& s) {
  for (double** p : {&s.H, &s.S, &s.T, &s.Hs64, &s.P64, &s.C64, &s.HW, &s.SW, &s.H1, &s.S1, &s.H2,
                     &s.S2, &s.partials, &s.trace, &s.HC64, &s.SC64, &s.G0_64, &s.G1_64, &s.PG64,
                     &s.D64, &s.HD64, &s.SD64})
    bfree(*p);
  for (float** p : {&s.Hs, &s.S32, &s.P, &s.C, &s.HC, &s.SC, &s.G0, &s.G1, &s.PG, &s.D, &s.HD,
                    &s.SD})
    bfree(*p);
}

bool host_symmetric(const double* A, int64_t n, bool* finite) {
  *finite = true;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i; j < n; ++j) {
      const double a = A[i * n + j], c = A[j * n + i];
      if (!std::isfinite(a) || !std::isfinite(c)) {
        *finite = false;
        return false;
      }
      if (!(fabs(a - c) <= 1e-10 * fmax(1.0, fmax(fabs(a), fabs(c))))) return false;
    }
  return true;
}

int alloc_sys_work(omm_batch* b, BSys& s, int max_iter, bool need32, bool need64) {
  const size_t mn = (size_t)s.M * s.N, mm = (size_t)s.M * s.M, nn = (size_t)s.N * s.N;
  BTRY(balloc(b, &s.Hs64, nn));
  BTRY(balloc(b, &s.C64, mn));
  if (need32) {
    BTRY(balloc(b, &s.Hs, nn));
    BTRY(balloc(b, &s.S32, nn));
    for (float** p : {&s.C, &s.HC, &s.SC, &s.G0, &s.G1, &s.PG, &s.D, &s.HD, &s.SD})
      BTRY(balloc(b, p, mn));
  }
  if (need64)
    for (double** p : {&s.HC64, &s.SC64, &s.G0_64, &s.G1_64, &s.PG64, &s.D64, &s.HD64, &s.SD64})
      BTRY(balloc(b, p, mn));
  for (double** p : {&s.HW, &s.SW, &s.H1, &s.S1, &s.H2, &s.S2}) BTRY(balloc(b, p, mm));
  BTRY(balloc(b, &s.partials, (size_t)GROUP_BLOCKS * NCOEF));
  if (s.trace_cap < max_iter + 2) {
    bfree(s.trace);
    BTRY(balloc(b, &s.trace, (size_t)max_iter + 2));
    s.trace_cap = max_iter + 2;
  }
  return OMM_OK;
}

// Shift, preconditioner (FP64 Gauss-Jordan) and FP32 operator copies of one system.
int setup_sys(omm_batch* b, BSys& s, double eta, double tau, bool need32) {
  const int64_t nn = s.N * s.N;
  BHIP(b, shift_hamiltonian(s.H, s.S, eta, s.Hs64, nn, b->stream));
  if (need32) {
    BHIP(b, convert_f64_f32(s.Hs64, s.Hs, nn, b->stream));
    BHIP(b, convert_f64_f32(s.S, s.S32, nn, b->stream));
  }
  const int kind = !(tau > 0.0) ? 0 : (isinf(tau) ? 1 : 2);
  if (kind == 2 && !s.have_T) return bfail(b, OMM_E_ARG, "a finite tau > 0 needs T");
  if (kind != s.p_kind || (kind == 2 && tau != s.p_tau)) {
    if (kind > 0) {
      BTRY(balloc(b, &s.P64, (size_t)nn));
      if (kind == 1) BHIP(b, copy_f64(s.S, s.P64, nn, b->stream));
      else BHIP(b, axpby_f64(s.S, s.T, s.P64, 1.0, 1.0 / tau, nn, b->stream));
      const size_t need = std::max(invert_work_doubles(s.N), inverse_residual_work_doubles(s.N));
      if (need > b->inv_cap) {
        bfree(b->inv_work);
        BTRY(balloc(b, &b->inv_work, need));
        b->inv_cap = need;
      }
      int bad = 0;
      BHIP(b, invert_in_place(s.P64, s.N, b->inv_work, b->stream, &bad));
      if (bad) {
        s.p_kind = -1;
        return bfail(b, OMM_E_PRECON, "preconditioner inversion hit a singular pivot block or a "
                                      "non-finite value");
      }
      BHIP(b, symmetrize(s.P64, s.N, b->stream));
      double res = 0.0;
      BHIP(b, inverse_residual(s.P64, s.S, kind == 2 ? s.T : nullptr, 1.0 / tau, s.N, b->inv_work,
                               b->stream, &res));
      if (!(res <= INVERSE_RESIDUAL_LIMIT)) {
        s.p_kind = -1;
        return bfail(b, OMM_E_PRECON, "preconditioner inverse is inaccurate (probe residual " +
                                          std::to_string(res) + ")");
      }
    }
    s.p_kind = kind;
    s.p_tau = tau;
    s.p32_valid = false;
  }
  if (s.p_kind > 0 && need32 && !s.p32_valid) {
    BTRY(balloc(b, &s.P, (size_t)nn));
    BHIP(b, convert_f64_f32(s.P64, s.P, nn, b->stream));
    s.p32_valid = true;
  }
  return OMM_OK;
}

GemmOp gop(int M, int N, int K, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
           int64_t ldc, double alpha = 1.0, const void* X = nullptr, int64_t ldx = 0,
           double beta = 0.0) {
  GemmOp op{};
  op.M = M; op.N = N; op.nseg = 1;
  op.A[0] = A; op.lda[0] = lda;
  op.B[0] = B; op.ldb[0] = ldb;
  op.K[0] = K;
  op.C = C; op.ldc = ldc;
  op.X = X; op.ldx = ldx;
  op.alpha = alpha; op.beta = beta;
  return op;
}

// Tile prefix sums for `tile`, uploaded with the op list; grid = min(tiles, 2 per CU).
int upload_list(omm_batch* b, OpList& L, int tile) {
  const int n = (int)L.ops.size();
  if (n == 0) return OMM_OK;
  if (L.cap < n) {
    free_list(L);
    BTRY(balloc(b, &L.d_ops, (size_t)n));
    BTRY(balloc(b, &L.d_tiles, (size_t)n + 1));
    if (hipMalloc((void**)&L.d_done, n * sizeof(int*)) != hipSuccess)
      return bfail(b, OMM_E_ALLOC, "hipMalloc failed");
    L.cap = n;
  }
  std::vector<int> ts(n + 1, 0);
  const int bm = gemm_tile_rows(tile, L.d.compute), bn = gemm_tile_cols(tile, L.d.compute);
  for (int i = 0; i < n; ++i)
    ts[i + 1] = ts[i] + ((L.ops[i].M + bm - 1) / bm) * ((L.ops[i].N + bn - 1) / bn);
  L.d.tile = tile;
  L.d.splitk = 1;
  L.grid = std::min(ts[n], 512);
  BHIP(b, hipMemcpyAsync(L.d_ops, L.ops.data(), n * sizeof(GemmOp), hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipMemcpyAsync(L.d_tiles, ts.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipMemcpyAsync((void*)L.d_done, L.done.data(), n * sizeof(int*), hipMemcpyHostToDevice,
                         b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  return OMM_OK;
}

int launch_list(omm_batch* b, OpList& L) {
  if (L.ops.empty()) return OMM_OK;
  BHIP(b, gemm_grouped_launch(L.d, L.d_ops, L.d_tiles, L.d_done, (int)L.ops.size(), L.grid,
                              b->stream));
  return OMM_OK;
}

// Times the grouped launch with each macro tile once (after a warm-up) and keeps the fastest.
int tune_list(omm_batch* b, OpList& L) {
  if (L.ops.empty() || L.tuned) return OMM_OK;
  hipEvent_t e0, e1;
  BHIP(b, hipEventCreate(&e0));
  BHIP(b, hipEventCreate(&e1));
  float best = 1e30f;
  int best_t = 0;
  for (int t = 0; t < gemm_grouped_num_tiles(); ++t) {
    BTRY(upload_list(b, L, t));
    BTRY(launch_list(b, L));
    BHIP(b, hipEventRecord(e0, b->stream));
    BTRY(launch_list(b, L));
    BHIP(b, hipEventRecord(e1, b->stream));
    BHIP(b, hipEventSynchronize(e1));
    float ms = 0.f;
    BHIP(b, hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      best_t = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  BTRY(upload_list(b, L, best_t));
  L.tuned = true;
  return OMM_OK;
}

// Builds the op lists of every CG stage of one phase (FP32 or FP64) from the current buffers.
int build_lists(omm_batch* b, bool f64) {
  PhaseLists& L = f64 ? b->L64 : b->L32;
  for (OpList* l : L.all()) {
    l->ops.clear();
    l->done.clear();
    l->tuned = false;
  }
  const int cm = f64 ? CF64 : CF32, tw = f64 ? T_F64 : T_F32;
  L.init1.d = GemmDesc{cm, tw, tw, tw, tw, KC, KC, 0, 1};
  L.init2.d = GemmDesc{cm, tw, tw, T_F64, T_F64, KC, KC, 0, 1};
  for (int p = 0; p < 2; ++p) {
    L.grad[p].d = GemmDesc{cm, T_F64, tw, tw, tw, KC, RC, 0, 1};
    L.pg[p].d = GemmDesc{cm, tw, tw, tw, tw, KC, KC, 0, 1};
  }
  L.hdsd.d = GemmDesc{cm, tw, tw, tw, tw, KC, KC, 0, 1};
  L.proj.d = GemmDesc{cm, tw, tw, T_F64, T_F64, KC, KC, 0, 1};
  for (size_t i = 0; i < b->sys.size(); ++i) {
    BSys& s = b->sys[i];
    const int M = (int)s.M, N = (int)s.N;
    // M x N state and products, and the operators, of the phase's precision
    void *C, *HC, *SC, *G0, *G1, *PG, *D, *HD, *SD;
    const void *Hs, *S, *P;
    if (f64) {
      C = s.C64; HC = s.HC64; SC = s.SC64; G0 = s.G0_64; G1 = s.G1_64; PG = s.PG64;
      D = s.D64; HD = s.HD64; SD = s.SD64; Hs = s.Hs64; S = s.S; P = s.P64;
    } else {
      C = s.C; HC = s.HC; SC = s.SC; G0 = s.G0; G1 = s.G1; PG = s.PG;
      D = s.D; HD = s.HD; SD = s.SD; Hs = s.Hs; S = s.S32; P = s.P;
    }
    // complex systems (real embeddings): every product follows C's row pairs and is computed
    // for its first M / 2 rows (group_pair_rows fills the rest)
    const int Mo = b->cplx ? M / 2 : M;
    const int* dn = &b->st[i].done;
    L.init1.ops.push_back(gop(Mo, N, N, C, N, Hs, N, HC, N));
    L.init1.ops.push_back(gop(Mo, N, N, C, N, S, N, SC, N));
    L.init2.ops.push_back(gop(Mo, M, N, HC, N, C, N, s.HW, M));
    L.init2.ops.push_back(gop(Mo, M, N, SC, N, C, N, s.SW, M));
    for (int k = 0; k < 2; ++k) L.init1.done.push_back(nullptr), L.init2.done.push_back(nullptr);
    for (int p = 0; p < 2; ++p) {
      void* G = p ? G1 : G0;
      GemmOp g = gop(Mo, N, M, s.HW, M, SC, N, G, N, -4.0, HC, N, 8.0);
      g.nseg = 2;
      g.A[1] = s.SW; g.lda[1] = M;
      g.B[1] = HC; g.ldb[1] = N;
      g.K[1] = M;
      L.grad[p].ops.push_back(g);
      L.grad[p].done.push_back(dn);
      if (s.p_kind > 0) {
        L.pg[p].ops.push_back(gop(Mo, N, N, G, N, P, N, PG, N));
        L.pg[p].done.push_back(dn);
      }
    }
    L.hdsd.ops.push_back(gop(Mo, N, N, D, N, Hs, N, HD, N));
    L.hdsd.ops.push_back(gop(Mo, N, N, D, N, S, N, SD, N));
    for (int k = 0; k < 2; ++k) L.hdsd.done.push_back(dn);
    L.proj.ops.push_back(gop(Mo, M, N, D, N, HC, N, s.H1, M));
    L.proj.ops.push_back(gop(Mo, M, N, D, N, SC, N, s.S1, M));
    L.proj.ops.push_back(gop(Mo, M, N, D, N, HD, N, s.H2, M));
    L.proj.ops.push_back(gop(Mo, M, N, D, N, SD, N, s.S2, M));
    for (int k = 0; k < 4; ++k) L.proj.done.push_back(dn);
  }
  for (OpList* l : L.all()) BTRY(upload_list(b, *l, 1));
  return OMM_OK;
}

// Complex batches: the second half of the rows of the products named by `which` (see
// group_pair_rows).
int fill_pairs(omm_batch* b, const SysDev* d_sys, int which, int parity, bool check_done) {
  if (!b->cplx) return OMM_OK;
  int mm = 0, mn = 0;
  for (const BSys& s : b->sys) {
    mm = std::max(mm, (int)s.M);
    mn = std::max(mn, (int)s.N);
  }
  BHIP(b, group_pair_rows(d_sys, (int)b->sys.size(), which, parity, check_done, mm, mn,
                          b->stream));
  return OMM_OK;
}

// One line search of every live system (k = line-search index: parity of G, first flag).
int batch_iteration(omm_batch* b, PhaseLists& L, const SysDev* d_sys, int k) {
  const int n = (int)b->sys.size();
  const int p = k & 1;
  BTRY(launch_list(b, L.grad[p]));
  BTRY(fill_pairs(b, d_sys, 2, p, true));
  BTRY(launch_list(b, L.pg[p]));
  BTRY(fill_pairs(b, d_sys, 3, p, true));
  BHIP(b, group_direction(d_sys, n, p, k == 0 ? 1 : 0, b->stream));
  BTRY(launch_list(b, L.hdsd));
  BTRY(fill_pairs(b, d_sys, 4, p, true));
  BTRY(launch_list(b, L.proj));
  BTRY(fill_pairs(b, d_sys, 5, p, true));
  BHIP(b, group_line_search(d_sys, n, b->stream));
  BHIP(b, group_update(d_sys, n, b->stream));
  return OMM_OK;
}

void drop_graph(omm_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

int read_states(omm_batch* b) {
  BHIP(b, hipMemcpyAsync(b->st_host, b->st, b->sys.size() * sizeof(DevState),
                         hipMemcpyDeviceToHost, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  return OMM_OK;
}

// Device descriptors of every system for one phase.
int upload_sysdev(omm_batch* b, bool f64) {
  const int n = (int)b->sys.size();
  std::vector<SysDev> sd(n);
  for (int i = 0; i < n; ++i) {
    BSys& s = b->sys[i];
    if (f64)
      sd[i] = SysDev{s.C64, s.HC64, s.SC64, s.G0_64, s.G1_64, s.PG64, s.D64, s.HD64, s.SD64,
                     s.HW, s.SW, s.H1, s.S1, s.H2, s.S2, s.partials, b->st + i, s.trace, (int)s.M,
                     (int)s.N, s.p_kind > 0 ? 1 : 0, b->cplx ? 1 : 0, 1};
    else
      sd[i] = SysDev{s.C, s.HC, s.SC, s.G0, s.G1, s.PG, s.D, s.HD, s.SD, s.HW, s.SW, s.H1, s.S1,
                     s.H2, s.S2, s.partials, b->st + i, s.trace, (int)s.M, (int)s.N,
                     s.p_kind > 0 ? 1 : 0, b->cplx ? 1 : 0, 0};
  }
  BHIP(b, hipMemcpyAsync(f64 ? b->d_sys64 : b->d_sys, sd.data(), n * sizeof(SysDev),
                         hipMemcpyHostToDevice, b->stream));
  return OMM_OK;
}

// One CG phase of every system from its current C (of the phase's precision): initial products,
// E_0, then up to max_iter line searches, each system stopping on its own (Eq. 18 with tol).
int run_phase(omm_batch* b, bool f64, double tol, int max_iter) {
  const int n = (int)b->sys.size();
  PhaseLists& L = f64 ? b->L64 : b->L32;
  const SysDev* d_sys = f64 ? b->d_sys64 : b->d_sys;
  for (int i = 0; i < n; ++i) {
    DevState& h = b->st_host[i];
    h = DevState{};
    h.tol = tol;
    h.max_iter = max_iter;
  }
  BHIP(b, hipMemcpyAsync(b->st, b->st_host, n * sizeof(DevState), hipMemcpyHostToDevice, b->stream));
  drop_graph(b);
  BTRY(upload_sysdev(b, f64));
  BTRY(build_lists(b, f64));

  // initial products and E_0 of every system
  BTRY(tune_list(b, L.init1));
  BTRY(launch_list(b, L.init1));
  BTRY(fill_pairs(b, d_sys, 0, 0, false));
  BTRY(tune_list(b, L.init2));
  BTRY(launch_list(b, L.init2));
  BTRY(fill_pairs(b, d_sys, 1, 0, false));
  BHIP(b, group_energy_init(d_sys, n, b->stream));
  BTRY(read_states(b));
  bool all_done = true;
  for (int i = 0; i < n; ++i) all_done = all_done && b->st_host[i].done != 0;
  if (max_iter > 0 && !all_done) {
    // first line search eagerly (autotunes each grouped product while every system is live)
    BTRY(tune_list(b, L.grad[0]));
    BTRY(tune_list(b, L.pg[0]));
    L.grad[1].d.tile = L.grad[0].d.tile;
    L.pg[1].d.tile = L.pg[0].d.tile;
    BTRY(upload_list(b, L.grad[1], L.grad[0].d.tile));
    BTRY(upload_list(b, L.pg[1], L.pg[0].d.tile));
    BTRY(launch_list(b, L.grad[0]));
    BTRY(fill_pairs(b, d_sys, 2, 0, true));
    BTRY(launch_list(b, L.pg[0]));
    BTRY(fill_pairs(b, d_sys, 3, 0, true));
    BHIP(b, group_direction(d_sys, n, 0, 1, b->stream));
    BTRY(tune_list(b, L.hdsd));
    BTRY(launch_list(b, L.hdsd));
    BTRY(fill_pairs(b, d_sys, 4, 0, true));
    BTRY(tune_list(b, L.proj));
    BTRY(launch_list(b, L.proj));
    BTRY(fill_pairs(b, d_sys, 5, 0, true));
    BHIP(b, group_line_search(d_sys, n, b->stream));
    BHIP(b, group_update(d_sys, n, b->stream));
    // line searches 1 and 2 (parities 1, 0) captured once, replayed until all systems stop
    BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int r1 = batch_iteration(b, L, d_sys, 1);
    int r2 = r1 == OMM_OK ? batch_iteration(b, L, d_sys, 2) : r1;
    hipGraph_t g = nullptr;
    hipError_t ec = hipStreamEndCapture(b->stream, &g);
    if (r1 != OMM_OK || r2 != OMM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return r1 != OMM_OK ? r1 : r2;
    }
    BHIP(b, ec);
    b->graph = g;
    BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    const int launches = (max_iter + 1) / 2;
    for (int l = 0; l < launches; ++l) {
      BHIP(b, hipGraphLaunch(b->exec, b->stream));
      if ((l + 1) % 4 == 0 || l + 1 == launches) {
        BTRY(read_states(b));
        all_done = true;
        for (int i = 0; i < n; ++i) all_done = all_done && b->st_host[i].done != 0;
        if (all_done) break;
      }
    }
  }
  BTRY(read_states(b));
  for (int i = 0; i < n; ++i) {
    const DevState& h = b->st_host[i];
    if (h.done < 0)
      return bfail(b, h.done, "system " + std::to_string(i) + " stopped with error " +
                                  std::to_string(h.done) + (f64 ? " (FP64 phase)" : " (FP32 phase)"));
  }
  return OMM_OK;
}

}  // namespace

extern "C" {

int omm_batch_create(int nsys, const int64_t* N, const int64_t* M, omm_batch** out) {
  if (!out) return OMM_E_ARG;
  *out = nullptr;
  if (nsys <= 0 || !N || !M) return OMM_E_ARG;
  for (int i = 0; i < nsys; ++i)
    if (N[i] <= 0 || M[i] <= 0 || M[i] > N[i] || N[i] > (1 << 16)) return OMM_E_ARG;
  omm_batch* b = new omm_batch();
  b->sys.resize(nsys);
  for (int i = 0; i < nsys; ++i) {
    b->sys[i].N = N[i];
    b->sys[i].M = M[i];
  }
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc((void**)&b->st, nsys * sizeof(DevState)) != hipSuccess ||
      hipHostMalloc((void**)&b->st_host, nsys * sizeof(DevState), 0) != hipSuccess ||
      hipMalloc((void**)&b->d_sys, nsys * sizeof(SysDev)) != hipSuccess ||
      hipMalloc((void**)&b->d_sys64, nsys * sizeof(SysDev)) != hipSuccess) {
    omm_batch_destroy(b);
    return OMM_E_HIP;
  }
  b->iters.assign(nsys, 0);
  b->E.assign(nsys, 0.0);
  *out = b;
  return OMM_OK;
}

int omm_batch_destroy(omm_batch* b) {
  if (!b) return OMM_E_ARG;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  for (BSys& s : b->sys) free_sys(s);
  for (OpList* L : b->L32.all()) free_list(*L);
  for (OpList* L : b->L64.all()) free_list(*L);
  bfree(b->st);
  bfree(b->d_sys);
  bfree(b->d_sys64);
  bfree(b->inv_work);
  bfree(b->d_cmp);
  if (b->st_host) (void)hipHostFree(b->st_host);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return OMM_OK;
}

namespace {
// omm_batch_set_HS and omm_batch_set_HS_device: validation (on the host, or by a kernel for
// device inputs), then S and T compared with the stored copies, then H.
int batch_set_HS(omm_batch* b, int i, const double* H, const double* S, const double* T,
                 bool host) {
  if (!b) return OMM_E_ARG;
  if (i < 0 || i >= (int)b->sys.size()) return bfail(b, OMM_E_ARG, "system index out of range");
  if (!H || !S) return bfail(b, OMM_E_ARG, "H and S are required");
  BSys& s = b->sys[i];
  const int64_t n = s.N;
  const size_t nn = (size_t)n * n;
  BTRY(balloc(b, &b->d_cmp, 2));
  const double* mats[3] = {H, S, T};
  for (int k = 0; k < 3; ++k) {
    if (!mats[k]) continue;
    bool fin = true, sym = true;
    if (host) {
      sym = host_symmetric(mats[k], n, &fin);
    } else {
      int h[2] = {0, 0};
      BHIP(b, hipMemsetAsync(b->d_cmp, 0, 2 * sizeof(int), b->stream));
      BHIP(b, validate_symmetric(mats[k], n, 1e-10, b->d_cmp, b->stream));
      BHIP(b, hipMemcpyAsync(h, b->d_cmp, 2 * sizeof(int), hipMemcpyDeviceToHost, b->stream));
      BHIP(b, hipStreamSynchronize(b->stream));
      fin = h[0] == 0;
      sym = fin && h[1] == 0;
    }
    if (!sym)
      return bfail(b, fin ? OMM_E_ASYMMETRIC : OMM_E_NONFINITE,
                   "system " + std::to_string(i) + ": input not finite/symmetric");
  }
  const hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  BTRY(balloc(b, &s.H, nn));
  BTRY(balloc(b, &s.S, nn));
  BTRY(balloc(b, &s.Hs64, nn));
  if (T) BTRY(balloc(b, &s.T, nn));
  // S and T go in through Hs (rebuilt from H and S by the next setup) and are compared with the
  // stored copies: when neither changed bit for bit (an SCF step at a fixed geometry) the
  // system keeps its preconditioner.
  const bool compare = s.have_HS && (T != nullptr) == s.have_T;
  const int kept_kind = s.p_kind;
  // until the new inputs are all in: a failure below leaves the system without inputs and
  // without a preconditioner
  s.have_HS = false;
  s.p_kind = -1;
  int diff = compare ? 0 : 1;
  BHIP(b, hipMemcpyAsync(b->d_cmp, &diff, sizeof(int), hipMemcpyHostToDevice, b->stream));
  double* dsts[2] = {s.S, s.T};
  const double* srcs[2] = {S, T};
  for (int k = 0; k < 2; ++k) {
    if (!srcs[k]) continue;
    BHIP(b, hipMemcpyAsync(s.Hs64, srcs[k], nn * sizeof(double), kind, b->stream));
    BHIP(b, symmetrize(s.Hs64, n, b->stream));
    BHIP(b, copy_compare_f64(s.Hs64, dsts[k], (int64_t)nn, b->d_cmp, b->stream));
  }
  BHIP(b, hipMemcpyAsync(&diff, b->d_cmp, sizeof(int), hipMemcpyDeviceToHost, b->stream));
  BHIP(b, hipMemcpyAsync(s.H, H, nn * sizeof(double), kind, b->stream));
  BHIP(b, symmetrize(s.H, n, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  s.have_T = T != nullptr;
  s.have_HS = true;
  if (!diff) s.p_kind = kept_kind;
  drop_graph(b);
  return OMM_OK;
}
}  // namespace

int omm_batch_set_HS(omm_batch* b, int i, const double* H, const double* S, const double* T) {
  return batch_set_HS(b, i, H, S, T, true);
}

int omm_batch_set_HS_device(omm_batch* b, int i, const double* dH, const double* dS,
                            const double* dT) {
  return batch_set_HS(b, i, dH, dS, dT, false);
}

int omm_batch_set_precision(omm_batch* b, int mode, int fp64_refine) {
  if (!b) return OMM_E_ARG;
  if (mode != OMM_FP32 && mode != OMM_FP64)
    return bfail(b, OMM_E_ARG, "batched systems run OMM_FP32 or OMM_FP64 products");
  b->mode = mode;
  b->refine = mode == OMM_FP32 && fp64_refine != 0;
  return OMM_OK;
}

int omm_batch_set_mixed_tol(omm_batch* b, double tol) {
  if (!b) return OMM_E_ARG;
  if (!(tol >= 0.0)) return bfail(b, OMM_E_ARG, "need tol >= 0");
  b->mixed_tol = tol;
  return OMM_OK;
}

int omm_batch_minimize(omm_batch* b, const double* const* C0, const double* eta, const double* tau,
                       double tol, int max_iter) {
  if (!b || !eta || !tau) return b ? bfail(b, OMM_E_ARG, "eta and tau are required") : OMM_E_ARG;
  if (!(tol >= 0.0) || max_iter < 0) return bfail(b, OMM_E_ARG, "need tol >= 0, max_iter >= 0");
  const int n = (int)b->sys.size();
  const bool run32 = b->mode == OMM_FP32, run64 = b->mode == OMM_FP64 || b->refine;
  for (int i = 0; i < n; ++i) {
    BSys& s = b->sys[i];
    if (!s.have_HS) return bfail(b, OMM_E_STATE, "system " + std::to_string(i) + " has no H/S");
    if ((!C0 || !C0[i]) && !s.have_C)
      return bfail(b, OMM_E_STATE, "system " + std::to_string(i) + ": no C0 and no C to resume");
    BTRY(alloc_sys_work(b, s, max_iter, run32, run64));
    BTRY(setup_sys(b, s, eta[i], tau[i], run32));
    const size_t mn = (size_t)s.M * s.N;
    if (C0 && C0[i]) {
      BHIP(b, hipMemcpyAsync(s.C64, C0[i], mn * sizeof(double), hipMemcpyHostToDevice, b->stream));
      s.c64_current = true;
    }
    // the first phase starts from the latest C, converted to its precision
    if (run32 && s.c64_current) BHIP(b, convert_f64_f32(s.C64, s.C, (int64_t)mn, b->stream));
    if (!run32 && !s.c64_current) BHIP(b, convert_f32_f64(s.C, s.C64, (int64_t)mn, b->stream));
    s.have_C = true;
  }
  b->iters32.assign(n, 0);
  b->iters64.assign(n, 0);
  if (run32) {
    BTRY(run_phase(b, false, b->refine ? std::max(tol, b->mixed_tol) : tol, max_iter));
    for (int i = 0; i < n; ++i) {
      b->iters32[i] = b->st_host[i].iter;
      b->sys[i].c64_current = false;
    }
  }
  if (run64) {
    if (run32)  // the FP64 phase starts from the FP32 phase's C
      for (BSys& s : b->sys)
        BHIP(b, convert_f32_f64(s.C, s.C64, (int64_t)s.M * s.N, b->stream));
    BTRY(run_phase(b, true, tol, max_iter));
    for (int i = 0; i < n; ++i) {
      b->iters64[i] = b->st_host[i].iter;
      b->sys[i].c64_current = true;
    }
  }
  int worst = OMM_OK;
  for (int i = 0; i < n; ++i) {
    const DevState& h = b->st_host[i];
    b->iters[i] = b->iters32[i] + b->iters64[i];
    b->E[i] = h.E;
    if (h.done != 1) worst = OMM_W_MAXITER;
  }
  return worst;
}

int omm_batch_phase_iterations(omm_batch* b, int* iters32, int* iters64) {
  if (!b) return OMM_E_ARG;
  for (size_t i = 0; i < b->sys.size(); ++i) {
    if (iters32) iters32[i] = i < b->iters32.size() ? b->iters32[i] : 0;
    if (iters64) iters64[i] = i < b->iters64.size() ? b->iters64[i] : 0;
  }
  return OMM_OK;
}

int omm_batch_energy(omm_batch* b, double* E) {
  if (!b || !E) return OMM_E_ARG;
  for (size_t i = 0; i < b->E.size(); ++i) E[i] = b->E[i] * (b->cplx ? 0.5 : 1.0);
  return OMM_OK;
}

int omm_batch_create_complex(int nsys, const int64_t* N, const int64_t* M, omm_batch** out) {
  if (!out) return OMM_E_ARG;
  *out = nullptr;
  if (nsys <= 0 || !N || !M) return OMM_E_ARG;
  std::vector<int64_t> N2(nsys), M2(nsys);
  for (int i = 0; i < nsys; ++i) {
    if (N[i] <= 0 || M[i] <= 0 || M[i] > N[i] || N[i] > (1 << 15)) return OMM_E_ARG;
    N2[i] = 2 * N[i];
    M2[i] = 2 * M[i];
  }
  const int r = omm_batch_create(nsys, N2.data(), M2.data(), out);
  if (r != OMM_OK) return r;
  (*out)->cplx = true;
  (*out)->Nc.assign(N, N + nsys);
  (*out)->Mc.assign(M, M + nsys);
  return OMM_OK;
}

int omm_batch_set_HS_complex(omm_batch* b, int i, const double* H_re, const double* H_im,
                             const double* S_re, const double* S_im, const double* T_re,
                             const double* T_im) {
  if (!b) return OMM_E_ARG;
  if (!b->cplx) return bfail(b, OMM_E_STATE, "not a complex batch (omm_batch_create_complex)");
  if (i < 0 || i >= (int)b->sys.size()) return bfail(b, OMM_E_ARG, "system index out of range");
  if (!H_re || !S_re) return bfail(b, OMM_E_ARG, "the real parts of H and S are required");
  if (!T_re && T_im) return bfail(b, OMM_E_ARG, "T_im without T_re");
  std::vector<double> H, S, T;
  embed_operator(H_re, H_im, b->Nc[i], H);
  embed_operator(S_re, S_im, b->Nc[i], S);
  if (T_re) embed_operator(T_re, T_im, b->Nc[i], T);
  return omm_batch_set_HS(b, i, H.data(), S.data(), T_re ? T.data() : nullptr);
}

int omm_batch_minimize_complex(omm_batch* b, const double* const* C0_re,
                               const double* const* C0_im, const double* eta, const double* tau,
                               double tol, int max_iter) {
  if (!b) return OMM_E_ARG;
  if (!b->cplx) return bfail(b, OMM_E_STATE, "not a complex batch (omm_batch_create_complex)");
  const int n = (int)b->sys.size();
  std::vector<std::vector<double>> C(n);
  std::vector<const double*> ptr(n, nullptr);
  for (int i = 0; i < n; ++i) {
    if (!C0_re || !C0_re[i]) continue;
    embed_rows(C0_re[i], C0_im ? C0_im[i] : nullptr, b->Mc[i], b->Nc[i], C[i]);
    ptr[i] = C[i].data();
  }
  return omm_batch_minimize(b, ptr.data(), eta, tau, tol, max_iter);
}

int omm_batch_iterations(omm_batch* b, int* iters) {
  if (!b || !iters) return OMM_E_ARG;
  for (size_t i = 0; i < b->iters.size(); ++i) iters[i] = b->iters[i];
  return OMM_OK;
}

int omm_batch_get_C(omm_batch* b, int i, double* C) {
  if (!b || !C) return OMM_E_ARG;
  if (i < 0 || i >= (int)b->sys.size()) return bfail(b, OMM_E_ARG, "system index out of range");
  BSys& s = b->sys[i];
  if (!s.have_C || !s.C64) return bfail(b, OMM_E_STATE, "system has no C");
  const size_t mn = (size_t)s.M * s.N;
  if (!s.c64_current) {
    BHIP(b, convert_f32_f64(s.C, s.C64, (int64_t)mn, b->stream));
    s.c64_current = true;
  }
  BHIP(b, hipMemcpyAsync(C, s.C64, mn * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  return OMM_OK;
}

const char* omm_batch_last_error(const omm_batch* b) {
  if (!b) return "null batch";
  return b->err.c_str();
}

}  // extern "C"
