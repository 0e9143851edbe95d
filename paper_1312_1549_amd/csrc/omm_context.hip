// Runtime of one OMM minimization: device buffers, the precision plan, the per-iteration stage
// sequence and the C-ABI entry points declared in include/omm.h.
//
// One CG line search (Sec. 2.3) is this stage sequence on the context's stream:
//   G  = 8 HC - 4 HW SC - 4 SW HC                 gradient, Eq. 12 (two-segment GEMM + epilogue)
//   PG = G P                                      preconditioning, Eq. 17 (skipped when P = I)
//   beta, D = -PG + beta D                        Polak-Ribiere direction
//   [HD | SD] = D [Hs | S]                        operator products (dominant cost)
//   [H' S' H'' S''] = D [HC; SC; HD; SD]^T        projections, Eqs. 14-15 (one launch)
//   alpha_0..4, x                                 quartic coefficients, Eq. 13, and line minimum
//   C, HC, SC += x (D, HD, SD); HW, SW update     Eq. 16 and footnote
//   E_new, stopping test                          Eq. 8 and Eq. 18
// Every scalar stays on the device; the host reads the small state block every few iterations
// to learn whether the run has stopped (later iterations are launched but return at once).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/omm.h"
#include "omm_internal.h"

using namespace omm;

namespace {

template <typename T>
struct Work {
  T *C = nullptr, *HC = nullptr, *SC = nullptr, *G = nullptr, *Gp = nullptr, *PG = nullptr,
    *D = nullptr, *HD = nullptr, *SD = nullptr;
  // BF16 scheme with an FP64 state: G (both parities), PG, HD and SD held in FP32. Their
  // products accumulate in FP32, so the FP32 value is the product itself (the stream-K fix-up
  // sums parts in FP64 and rounds once; G = 8 HC - 4 (...) is formed in FP64 and rounded once);
  // the state C, HC, SC stays FP64 and D is exact in its bf16 plane.
  float *PGf = nullptr, *HDf = nullptr, *SDf = nullptr, *Gf = nullptr, *Gpf = nullptr;
};

// A bf16 hi/lo pair of planes (x = hi + lo) feeding the BF16x3 GEMMs.
struct Plane {
  unsigned short* hi = nullptr;
  unsigned short* lo = nullptr;
  int64_t ld = 0;  // row length (elements)
};

constexpr int NSTAGE = 7;  // gradient, PG, PR+direction, [HD|SD], projections, line search, updates

template <typename T>
constexpr int elem_type() {
  return sizeof(T) == 8 ? T_F64 : T_F32;
}

}  // namespace

struct omm_ctx {
  int64_t N = 0, M = 0;
  // complex Hermitian problem of Nc orbitals, Mc Wannier functions held as its exact real
  // embedding (N = 2 Nc, M = 2 Mc); energies are reported for the complex problem (E / 2)
  bool cplx = false;
  int64_t Nc = 0, Mc = 0;
  int device = 0;
  int mode = OMM_FP64;
  int refine = 1;
  double mixed_tol = 1e-9;
  hipStream_t own = nullptr, stream = nullptr;
  std::string err;

  // inputs and derived operators (FP64)
  double *H = nullptr, *S = nullptr, *T = nullptr, *Hs = nullptr, *P = nullptr;
  float *Hs32 = nullptr, *S32 = nullptr, *P32 = nullptr;
  bool have_HS = false, have_T = false;
  bool hs_valid = false, s32_valid = false;
  double hs_eta = 0.0;
  int p_kind = -1;  // -1 not built, 0 identity, 1 S^-1, 2 (S + T/tau)^-1
  double p_tau = 0.0;
  bool p32_valid = false, hs32_valid = false;

  Work<double> w64;
  Work<float> w32;
  // BF16x3 operand planes: operators (set up once) and per-iteration operands
  Plane Hs_p, S_p, P_p, C_p, HC_p, SC_p, G_p, D_p, HD_p, SD_p, HW_p, SW_p;
  Plane HCt_p, SCt_p;  // planes of HC^T, SC^T (N x M): k-contiguous B of the gradient
  bool hsp_valid = false, sp_valid = false, pp_valid = false;
  double *HW = nullptr, *SW = nullptr, *H1 = nullptr, *S1 = nullptr, *H2 = nullptr, *S2 = nullptr;
  double *partials = nullptr, *ws = nullptr;
  size_t ws_bytes = 0;
  DevState* st = nullptr;
  DevState* st_host = nullptr;  // pinned
  int* flags = nullptr;
  double* trace = nullptr;
  int trace_cap = 0;
  double* nn_scratch = nullptr;  // N x N FP64 (density / EDM / preconditioner work)
  double* inv_work = nullptr;
  // Cholesky-reduced flavour: S = L L^T, the CG runs on C~ = C L with H~ = L^-1 Hs L^-T (held in
  // Hs and its derived copies) and S~ = I
  int flavour = OMM_FLAVOUR_DENSE;
  double *L = nullptr, *Linv = nullptr;
  bool l_valid = false;
  bool hs_reduced = false;      // Hs (and its planes / FP32 copy) holds H~
  double* Corig = nullptr;      // M x N: C = C~ L^-1 for the outputs
  // block-sparse operator products (BF16 scheme, dense flavour): K-block lists of Hs and S
  bool sparse = false;
  int* kl_ptr[2] = {nullptr, nullptr};  // Hs, S: per 256-column tile, offsets into kl_idx
  int* kl_idx[2] = {nullptr, nullptr};
  bool kl_valid[2] = {false, false};
  double kl_density[2] = {1.0, 1.0};    // listed K blocks / all K blocks

  bool have_C = false;
  int c_prec = OMM_FP64;  // precision in which the current C lives
  int c_flavour = OMM_FLAVOUR_DENSE;  // coordinates of the current C (C~ = C L when reduced)
  // active CG phase (continued by omm_iterate)
  bool phase_active = false;
  int phase_prec = OMM_FP64;  // precision of the active phase
  bool phase_mixed64 = false; // active phase: BF16x3 products on an FP64 state (with resyncs)
  int resync_every = 80;      // line searches between FP64 resynchronizations
  int since_resync = 0;
  double resync_E = 0.0;      // FP64 energy at the last resynchronization
  double p_residual = -1.0;   // probe residual of the last preconditioner inverse
  std::vector<int> ck_iter;   // FP64-exact energies of the mixed scheme: (line search, E)
  std::vector<double> ck_E;
  int phase_k = 0;            // line searches launched in the active phase
  int trace_off = 0;          // offset of the active phase in the energy trace
  int iters_before = 0;       // line searches of earlier phases of the last minimize call
  // hipGraph of two line searches of the active phase (replayed after the first two)
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int graph_parity = -1;  // phase_k & 1 at capture
  // profiling: HIP events around each stage of every launched line search
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  double stage_ms[NSTAGE] = {0};
  int prof_iters = 0;
  double eta_last = 0.0;
  int iters = 0, trace_n = 0;
  double last_rel = 0.0;
  std::vector<double> trace_host;
};

namespace {

int fail(omm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, x)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      return fail(ctx, OMM_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_));       \
  } while (0)

template <typename P>
int dalloc(omm_ctx* c, P** p, size_t count) {
  if (*p) return OMM_OK;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(P));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(c, OMM_E_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return OMM_OK;
}

template <typename P>
void dfree(P*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

#define TRY(x)                  \
  do {                          \
    int r_ = (x);               \
    if (r_ != OMM_OK) return r_; \
  } while (0)

template <typename T>
int alloc_work(omm_ctx* c, Work<T>& w) {
  const size_t mn = (size_t)c->M * c->N;
  TRY(dalloc(c, &w.C, mn));
  TRY(dalloc(c, &w.HC, mn));
  TRY(dalloc(c, &w.SC, mn));
  TRY(dalloc(c, &w.G, mn));
  TRY(dalloc(c, &w.Gp, mn));
  TRY(dalloc(c, &w.PG, mn));
  TRY(dalloc(c, &w.D, mn));
  TRY(dalloc(c, &w.HD, mn));
  TRY(dalloc(c, &w.SD, mn));
  if (sizeof(T) == 8 && c->mode == OMM_BF16X3 && c->refine) {
    TRY(dalloc(c, &w.PGf, mn));
    TRY(dalloc(c, &w.HDf, mn));
    TRY(dalloc(c, &w.SDf, mn));
    TRY(dalloc(c, &w.Gf, mn));
    TRY(dalloc(c, &w.Gpf, mn));
  }
  return OMM_OK;
}

template <typename T>
void free_work(Work<T>& w) {
  dfree(w.C); dfree(w.HC); dfree(w.SC); dfree(w.G); dfree(w.Gp); dfree(w.PG); dfree(w.D);
  dfree(w.HD); dfree(w.SD);
  dfree(w.PGf); dfree(w.HDf); dfree(w.SDf); dfree(w.Gf); dfree(w.Gpf);
}

// Row length of a bf16 plane with `cols` columns: a multiple of 64 elements, so that every row
// starts on a 128-byte line and each 64-byte K chunk the GEMM tiles fetch is one aligned request
// (an unaligned chunk straddles two).
int64_t plane_ld(int64_t cols) { return (cols + 63) / 64 * 64; }

int alloc_plane(omm_ctx* c, Plane& p, int64_t rows, int64_t cols) {
  if (p.hi) return OMM_OK;
  p.ld = plane_ld(cols);
  const size_t n = (size_t)rows * p.ld;
  TRY(dalloc(c, &p.hi, n));
  TRY(dalloc(c, &p.lo, n));
  // never read before written; zeroed so that a missed split could not depend on stale memory
  HIPCHK(c, hipMemsetAsync(p.hi, 0, n * sizeof(unsigned short), c->stream));
  HIPCHK(c, hipMemsetAsync(p.lo, 0, n * sizeof(unsigned short), c->stream));
  return OMM_OK;
}

void free_plane(Plane& p) {
  dfree(p.hi);
  dfree(p.lo);
}

// ---- tile / split-K choice --------------------------------------------------------------------
// Heuristic: the largest macro tile that still yields >= 1 workgroup per CU, split-K when even
// the 64x64 tiling leaves CUs idle and K is long. The autotuner replaces it per shape.
void heuristic_tiling(GemmDesc& d, int M, int N, int K) {
  const int cus = 256;
  if ((d.compute == CF64 || d.compute == CF32) && (long)M * N <= 65536 && K <= 512) {
    d.tile = 7;  // one wave per 16 x 16 tile, no staging: a few launches' latency, not a K loop's
    d.splitk = 1;
    return;
  }
  const long t128 = (long)((M + 127) / 128) * ((N + 127) / 128);
  const long t64 = (long)((M + 63) / 64) * ((N + 63) / 64);
  d.tile = t128 >= cus ? 0 : 1;
  d.splitk = 1;
  const long tiles = d.tile == 0 ? t128 : t64;
  if (tiles < cus && K >= 1024) {
    int sk = (int)((2 * cus + tiles - 1) / tiles);
    const int kmax = K / 256;
    if (sk > kmax) sk = kmax;
    if (sk > 16) sk = 16;
    if (sk > 1) d.splitk = sk;
  }
}

struct TuneKey {
  int v[11];
  bool operator<(const TuneKey& o) const {
    for (int i = 0; i < 11; ++i)
      if (v[i] != o.v[i]) return v[i] < o.v[i];
    return false;
  }
};

std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;  // -> (tile, splitk)
bool g_tune_loaded = false;

const char* tune_cache_path() { return getenv("OMM_AUTOTUNE_CACHE"); }

bool autotune_enabled() {
  const char* e = getenv("OMM_AUTOTUNE");
  return !(e && e[0] == '0');
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = tune_cache_path();
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  TuneKey k;
  int t, sk;
  while (fscanf(f, "%d %d %d %d %d %d %d %d %d %d %d %d %d", &k.v[0], &k.v[1], &k.v[2], &k.v[3],
                &k.v[4], &k.v[5], &k.v[6], &k.v[7], &k.v[8], &k.v[9], &k.v[10], &t, &sk) == 13)
    g_tune[k] = {t, sk};
  fclose(f);
}

void tune_save_locked() {
  const char* path = tune_cache_path();
  if (!path) return;
  FILE* f = fopen(path, "w");
  if (!f) return;
  for (const auto& kv : g_tune) {
    for (int i = 0; i < 11; ++i) fprintf(f, "%d ", kv.first.v[i]);
    fprintf(f, "%d %d\n", kv.second.first, kv.second.second);
  }
  fclose(f);
}

void drop_graph(omm_ctx* c);

int ensure_ws(omm_ctx* c, const GemmDesc& d, const GemmOp* ops, int nops) {
  const size_t need = gemm_ws_bytes(d, ops, nops);
  if (need == 0) return OMM_OK;
  if (need > c->ws_bytes) {
    drop_graph(c);  // a captured graph holds the old workspace address
    dfree(c->ws);
    c->ws_bytes = 0;
    TRY(dalloc(c, &c->ws, need / sizeof(double) + 1));
    c->ws_bytes = need;
  }
  return OMM_OK;
}

// Times each candidate (tile, split-K) once after a warm-up launch, then the three fastest twice
// more, and returns the one with the lowest of its times (a single timing picked a tile 5-10 %
// slower than the best now and then).
int autotune(omm_ctx* c, GemmDesc d, GemmOp* ops, int nops, int K, std::pair<int, int>* best) {
  const int M = ops[0].M, N = ops[0].N;
  std::vector<std::pair<int, int>> cands;
  for (int t = 0; t < gemm_num_tiles(); ++t) {
    GemmDesc dt = d;
    dt.tile = t;
    dt.splitk = 1;
    if (!gemm_supported(dt)) continue;
    const int bm = gemm_tile_rows(t, d.compute), bn = gemm_tile_cols(t, d.compute);
    const long tiles = (long)((M + bm - 1) / bm) * ((N + bn - 1) / bn);
    // the one-wave tile re-reads its operands per 16 x 16 output tile: small products only
    if (t == 7 && (tiles > 4096 || K > 2048)) continue;
    if (tiles >= 32 || t == 1) cands.push_back({t, 1});
    for (int sk : {2, 4, 8, 16}) {
      dt.splitk = sk;
      if (gemm_supported(dt) && tiles * sk <= 4096 && tiles < 512 && K / sk >= 256)
        cands.push_back({t, sk});
    }
  }
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  auto time_one = [&](const std::pair<int, int>& cand, bool warm, float* ms) -> int {
    GemmDesc dt = d;
    dt.tile = cand.first;
    dt.splitk = cand.second;
    TRY(ensure_ws(c, dt, ops, nops));
    if (warm) HIPCHK(c, gemm_launch(dt, ops, nops, nullptr, c->ws, c->ws_bytes, c->stream));
    HIPCHK(c, hipEventRecord(e0, c->stream));
    HIPCHK(c, gemm_launch(dt, ops, nops, nullptr, c->ws, c->ws_bytes, c->stream));
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    HIPCHK(c, hipEventElapsedTime(ms, e0, e1));
    return OMM_OK;
  };
  std::vector<float> t_best(cands.size());
  for (size_t i = 0; i < cands.size(); ++i) TRY(time_one(cands[i], true, &t_best[i]));
  std::vector<size_t> order(cands.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return t_best[a] < t_best[b]; });
  for (size_t r = 0; r < 2; ++r)
    for (size_t q = 0; q < order.size() && q < 3; ++q) {
      float ms = 0.f;
      TRY(time_one(cands[order[q]], false, &ms));
      t_best[order[q]] = std::min(t_best[order[q]], ms);
    }
  *best = {-1, 1};
  float best_ms = 1e30f;
  for (size_t i = 0; i < cands.size(); ++i)
    if (t_best[i] < best_ms) {
      best_ms = t_best[i];
      *best = cands[i];
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return OMM_OK;
}

// One GEMM launch with a tuned (or heuristic) tiling. `tunable` is false for in-place updates,
// which must not be run more than once.
// OMM_TILE=<t> pins every GEMM that supports macro tile t to it (no split-K, no autotuning), and
// with t >= 4 the FP64 / FP32 GEMMs to tile 4: used to compare tile implementations against
// each other.
int forced_tile() {
  const char* e = getenv("OMM_TILE");
  return (e && e[0]) ? atoi(e) : -1;
}

int gemm(omm_ctx* c, GemmDesc d, GemmOp* ops, int nops, const int* done, bool tunable = true) {
  const int K = ops[0].K[0] + (ops[0].nseg > 1 ? ops[0].K[1] : 0);
  const int M = ops[0].M, N = ops[0].N;
  heuristic_tiling(d, M, N, K);
  const double flops = 2.0 * M * N * (double)K * nops;
  const int ft = forced_tile();
  GemmDesc df = d;
  df.tile = ft;
  df.splitk = 1;
  if (ops[0].kptr) {  // block-sparse B, no split: the direct-to-LDS tile for the BF16 modes,
                      // the 128 x 128 tile at two workgroups per CU for FP64 / FP32
    d.tile = is_bf16_mode(d.compute) ? 5 : 4;
    d.splitk = 1;
  } else if (ft >= 0 && gemm_supported(df)) {
    d = df;
  } else if (ft >= 4 && !is_bf16_mode(d.compute)) {
    // the BF16-only tiles pinned: FP64 / FP32 products take tile 4 without split, the tile of
    // their block-sparse form (so that pinned dense and sparse runs sum in the same order)
    d.tile = 4;
    d.splitk = 1;
  } else if (tunable && flops >= 2e9 && autotune_enabled()) {
    TuneKey key{{d.compute, d.ta, d.tb, d.tc, d.tx, d.la, d.lb, M, N, K, nops}};
    std::pair<int, int> choice{-1, 1};
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      tune_load_locked();
      auto it = g_tune.find(key);
      if (it != g_tune.end()) choice = it->second;
    }
    if (choice.first < 0) {
      TRY(autotune(c, d, ops, nops, K, &choice));
      if (choice.first >= 0) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[key] = choice;
        tune_save_locked();
      }
    }
    if (choice.first >= 0) {
      d.tile = choice.first;
      d.splitk = choice.second;
    }
  }
  TRY(ensure_ws(c, d, ops, nops));
  HIPCHK(c, gemm_launch(d, ops, nops, done, c->ws, c->ws_bytes, c->stream));
  return OMM_OK;
}

GemmOp make_op(int M, int N, int K, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
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

int compute_of(int mode) {
  return mode == OMM_FP64 ? CF64 : (mode == OMM_FP32 ? CF32 : CBF16X3);
}

bool host_check(const double* A, int64_t n, bool* finite_ok) {
  *finite_ok = true;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = i; j < n; ++j) {
      const double a = A[i * n + j], b = A[j * n + i];
      if (!std::isfinite(a) || !std::isfinite(b)) {
        *finite_ok = false;
        return false;
      }
      const double m = fmax(1.0, fmax(fabs(a), fabs(b)));
      if (!(fabs(a - b) <= 1e-10 * m)) return false;
    }
  }
  return true;
}

int ensure_inputs(omm_ctx* c) {
  const size_t nn = (size_t)c->N * c->N;
  TRY(dalloc(c, &c->H, nn));
  TRY(dalloc(c, &c->S, nn));
  return OMM_OK;
}

// New inputs end the active minimization. H changes with every omm_set_HS, and with it
// Hs = H - eta S (or H~), its planes, FP32 copy and K-block list. What derives from S and T
// alone (P, its planes and FP32 copy, the Cholesky factor, S's planes, FP32 copy and K-block
// list) stays valid when neither changed: an SCF loop that updates H at a fixed geometry keeps
// its preconditioner (Sec. 3 reuses the previous step's coefficients the same way).
void invalidate(omm_ctx* c, bool s_or_t_changed) {
  drop_graph(c);
  c->phase_active = false;
  c->phase_mixed64 = false;
  c->kl_valid[0] = false;
  c->hsp_valid = false;
  c->hs_valid = false;
  c->hs32_valid = false;
  if (!s_or_t_changed) return;
  c->l_valid = false;
  c->kl_valid[1] = false;
  c->sp_valid = false;
  c->pp_valid = false;
  c->s32_valid = false;
  c->p_kind = -1;
  c->p32_valid = false;
}

bool reduced(const omm_ctx* c) { return c->flavour == OMM_FLAVOUR_CHOLESKY; }

// K-block lists of an N x N operator for the block-sparse products (which = 0: Hs, 1: S).
int build_klist(omm_ctx* c, const double* B, int which) {
  if (c->kl_valid[which]) return OMM_OK;
  const int64_t n = c->N;
  const int nkb = (int)((n + SPARSE_BK - 1) / SPARSE_BK);
  const int nt = (int)((n + SPARSE_BN - 1) / SPARSE_BN);
  unsigned char* dflags = nullptr;
  TRY(dalloc(c, &dflags, (size_t)nkb * nt));
  HIPCHK(c, block_pattern(B, n, dflags, c->stream));
  std::vector<unsigned char> flags((size_t)nkb * nt);
  HIPCHK(c, hipMemcpyAsync(flags.data(), dflags, flags.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  dfree(dflags);
  std::vector<int> ptr(nt + 1, 0), idx;
  for (int t = 0; t < nt; ++t) {
    for (int kb = 0; kb < nkb; ++kb)
      if (flags[(size_t)t * nkb + kb]) idx.push_back(kb);
    ptr[t + 1] = (int)idx.size();
  }
  if (idx.empty()) idx.push_back(0);  // an all-zero operator still needs a valid array
  drop_graph(c);
  dfree(c->kl_ptr[which]);
  dfree(c->kl_idx[which]);
  TRY(dalloc(c, &c->kl_ptr[which], ptr.size()));
  TRY(dalloc(c, &c->kl_idx[which], idx.size()));
  HIPCHK(c, hipMemcpyAsync(c->kl_ptr[which], ptr.data(), ptr.size() * sizeof(int),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->kl_idx[which], idx.data(), idx.size() * sizeof(int),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->kl_density[which] = (double)ptr[nt] / ((double)nkb * nt);
  c->kl_valid[which] = true;
  return OMM_OK;
}

bool sparse_products(const omm_ctx* c) {
  return c->sparse && c->mode == OMM_BF16X3 && !reduced(c);
}

// S = L L^T and L^-1 for the Cholesky-reduced flavour (Sec. 2.4), once per S.
int prepare_cholesky(omm_ctx* c) {
  if (c->l_valid) return OMM_OK;
  const size_t nn = (size_t)c->N * c->N;
  TRY(dalloc(c, &c->L, nn));
  TRY(dalloc(c, &c->Linv, nn));
  TRY(dalloc(c, &c->inv_work, std::max(invert_work_doubles(c->N), cholesky_work_doubles())));
  HIPCHK(c, copy_f64(c->S, c->L, (int64_t)nn, c->stream));
  int bad = 0;
  HIPCHK(c, cholesky_in_place(c->L, c->N, c->inv_work, c->stream, &bad));
  if (bad) return fail(c, OMM_E_PRECON, "Cholesky factorization of S failed: S is not positive definite");
  HIPCHK(c, copy_f64(c->L, c->Linv, (int64_t)nn, c->stream));
  HIPCHK(c, invert_in_place(c->Linv, c->N, c->inv_work, c->stream, &bad));
  if (bad) return fail(c, OMM_E_PRECON, "inverting the Cholesky factor hit a zero or non-finite pivot");
  c->l_valid = true;
  return OMM_OK;
}

// Hs = H - eta S (Sec. 2.2, Eq. 9) and, for mixed modes, FP32 copies of Hs and S. In the
// Cholesky-reduced flavour Hs is replaced by H~ = L^-1 (H - eta S) L^-T.
int prepare_shift(omm_ctx* c, double eta) {
  const size_t nn = (size_t)c->N * c->N;
  const bool red = reduced(c);
  if (red) TRY(prepare_cholesky(c));
  if (!c->hs_valid || c->hs_eta != eta || c->hs_reduced != red) {
    TRY(dalloc(c, &c->Hs, nn));
    HIPCHK(c, shift_hamiltonian(c->H, c->S, eta, c->Hs, (int64_t)nn, c->stream));
    if (red) {
      const int N = (int)c->N;
      TRY(dalloc(c, &c->nn_scratch, nn));
      // X = L^-1 Hs (B(n, k) = Hs[k][n] = Hs[n][k]), then H~ = X L^-T (B(n, k) = L^-1[n][k])
      GemmDesc d{CF64, T_F64, T_F64, T_F64, T_F64, KC, KC, 0, 1};
      GemmOp op = make_op(N, N, N, c->Linv, N, c->Hs, N, c->nn_scratch, N);
      TRY(gemm(c, d, &op, 1, nullptr, true));
      GemmOp op2 = make_op(N, N, N, c->nn_scratch, N, c->Linv, N, c->Hs, N);
      TRY(gemm(c, d, &op2, 1, nullptr, true));
      HIPCHK(c, symmetrize(c->Hs, N, c->stream));
    }
    c->hs_valid = true;
    c->hs_eta = eta;
    c->hs_reduced = red;
    c->kl_valid[0] = false;
    drop_graph(c);  // a captured graph may hold the old Hs lists
    c->hs32_valid = false;
    c->hsp_valid = false;
  }
  if (c->mode == OMM_BF16X3) {
    if (!c->hsp_valid) {
      TRY(alloc_plane(c, c->Hs_p, c->N, c->N));
      HIPCHK(c, split_bf16(c->Hs, c->Hs_p.hi, c->Hs_p.lo, c->N, c->N, c->Hs_p.ld, nullptr,
                           c->stream));
      c->hsp_valid = true;
    }
    if (!c->sp_valid && !red) {
      TRY(alloc_plane(c, c->S_p, c->N, c->N));
      HIPCHK(c, split_bf16(c->S, c->S_p.hi, c->S_p.lo, c->N, c->N, c->S_p.ld, nullptr, c->stream));
      c->sp_valid = true;
    }
    if (sparse_products(c)) {
      TRY(build_klist(c, c->Hs, 0));
      TRY(build_klist(c, c->S, 1));
    }
  } else if (c->mode == OMM_FP32) {
    if (!c->hs32_valid) {
      TRY(dalloc(c, &c->Hs32, nn));
      HIPCHK(c, convert_f64_f32(c->Hs, c->Hs32, (int64_t)nn, c->stream));
      c->hs32_valid = true;
    }
    if (!c->s32_valid && !red) {
      TRY(dalloc(c, &c->S32, nn));
      HIPCHK(c, convert_f64_f32(c->S, c->S32, (int64_t)nn, c->stream));
      c->s32_valid = true;
    }
  }
  return OMM_OK;
}

// P = (S + T/tau)^-1, S^-1 or I (Sec. 2.4, Eq. 17), factorized once per (S, T, tau).
int prepare_precon(omm_ctx* c, double tau) {
  // the Cholesky-reduced flavour needs none: S~ = I, and CG on C~ is the S^-1-preconditioned CG
  int kind = reduced(c) || !(tau > 0.0) ? 0 : (isinf(tau) ? 1 : 2);
  if (kind == 2 && !c->have_T)
    return fail(c, OMM_E_ARG, "a finite tau > 0 needs the kinetic matrix T");
  const size_t nn = (size_t)c->N * c->N;
  if (c->p_kind != kind || (kind == 2 && c->p_tau != tau)) {
    if (kind > 0) {
      TRY(dalloc(c, &c->P, nn));
      if (kind == 1) HIPCHK(c, copy_f64(c->S, c->P, (int64_t)nn, c->stream));
      else HIPCHK(c, axpby_f64(c->S, c->T, c->P, 1.0, 1.0 / tau, (int64_t)nn, c->stream));
      TRY(dalloc(c, &c->inv_work, std::max(invert_work_doubles(c->N),
                                            inverse_residual_work_doubles(c->N))));
      int bad = 0;
      HIPCHK(c, invert_in_place(c->P, c->N, c->inv_work, c->stream, &bad));
      if (bad) {
        c->p_kind = -1;
        return fail(c, OMM_E_PRECON, "preconditioner inversion hit a singular pivot block or a "
                                     "non-finite value");
      }
      HIPCHK(c, symmetrize(c->P, c->N, c->stream));
      // the inverse is used only if it inverts: max |X P (S + T/tau) - X| on +-1 probe rows
      double res = 0.0;
      HIPCHK(c, inverse_residual(c->P, c->S, kind == 2 ? c->T : nullptr, 1.0 / tau, c->N,
                                 c->inv_work, c->stream, &res));
      c->p_residual = res;
      if (!(res <= INVERSE_RESIDUAL_LIMIT)) {
        c->p_kind = -1;
        return fail(c, OMM_E_PRECON, "preconditioner inverse is inaccurate (probe residual " +
                                         std::to_string(res) + "): S + T/tau is near singular");
      }
    }
    c->p_kind = kind;
    c->p_tau = tau;
    c->p32_valid = false;
    c->pp_valid = false;
  }
  if (kind > 0 && c->mode == OMM_BF16X3 && !c->pp_valid) {
    TRY(alloc_plane(c, c->P_p, c->N, c->N));
    HIPCHK(c, split_bf16(c->P, c->P_p.hi, c->P_p.lo, c->N, c->N, c->P_p.ld, nullptr, c->stream));
    c->pp_valid = true;
  }
  if (kind > 0 && c->mode == OMM_FP32 && !c->p32_valid) {
    TRY(dalloc(c, &c->P32, nn));
    HIPCHK(c, convert_f64_f32(c->P, c->P32, (int64_t)nn, c->stream));
    c->p32_valid = true;
  }
  return OMM_OK;
}

int alloc_common(omm_ctx* c) {
  const size_t mm = (size_t)c->M * c->M;
  TRY(dalloc(c, &c->HW, mm));
  TRY(dalloc(c, &c->SW, mm));
  TRY(dalloc(c, &c->H1, mm));
  TRY(dalloc(c, &c->S1, mm));
  TRY(dalloc(c, &c->H2, mm));
  TRY(dalloc(c, &c->S2, mm));
  TRY(dalloc(c, &c->partials, (size_t)RED_BLOCKS * NCOEF));
  TRY(dalloc(c, &c->st, 1));
  if (!c->st_host) {
    if (hipHostMalloc((void**)&c->st_host, sizeof(DevState), 0) != hipSuccess) {
      c->st_host = nullptr;
      return fail(c, OMM_E_ALLOC, "hipHostMalloc failed");
    }
  }
  return OMM_OK;
}

// Operand of a GEMM: plain pointer, or the hi/lo planes for BF16x3; ld = row length.
struct Opnd {
  const void* p;
  const void* lo;
  int64_t ld;
};

GemmOp make_op2(int M, int N, int K, Opnd A, Opnd B, void* C, int64_t ldc, double alpha = 1.0,
                const void* X = nullptr, int64_t ldx = 0, double beta = 0.0) {
  GemmOp op = make_op(M, N, K, A.p, A.ld, B.p, B.ld, C, ldc, alpha, X, ldx, beta);
  op.Alo[0] = A.lo;
  op.Blo[0] = B.lo;
  return op;
}

Opnd pl(const Plane& p) { return {p.hi, p.lo, p.ld}; }
template <typename T>
Opnd dn(const T* p, int64_t ld) { return {p, nullptr, ld}; }

// The output planes an op's epilogue writes (the next product's operand).
void out_planes(GemmOp& op, const Plane& p) {
  op.Chi = p.hi;
  op.Clo = p.lo;
  op.ldp = p.ld;
}

// Planes for the per-iteration BF16x3 operands (M x N, N x M and M x M).
int alloc_iter_planes(omm_ctx* c) {
  for (Plane* p : {&c->C_p, &c->HC_p, &c->SC_p, &c->G_p, &c->D_p, &c->HD_p, &c->SD_p})
    TRY(alloc_plane(c, *p, c->M, c->N));
  TRY(alloc_plane(c, c->HCt_p, c->N, c->M));
  TRY(alloc_plane(c, c->SCt_p, c->N, c->M));
  TRY(alloc_plane(c, c->HW_p, c->M, c->M));
  TRY(alloc_plane(c, c->SW_p, c->M, c->M));
  return OMM_OK;
}

// Planes of a rows x cols array.
template <typename T>
int split(omm_ctx* c, const T* src, Plane& p, int64_t rows, int64_t cols, bool check_done = true) {
  HIPCHK(c, split_bf16(src, p.hi, p.lo, rows, cols, p.ld, check_done ? c->st : nullptr, c->stream));
  return OMM_OK;
}

// Planes of HC, SC and of their transposes (after every change of HC, SC).
template <typename T>
int split_state(omm_ctx* c, const T* HC, const T* SC, bool check_done = true) {
  const int M = (int)c->M, N = (int)c->N;
  const DevState* st = check_done ? c->st : nullptr;
  TRY(split(c, HC, c->HC_p, M, N, check_done));
  TRY(split(c, SC, c->SC_p, M, N, check_done));
  HIPCHK(c, split_bf16_t(HC, c->HCt_p.hi, c->HCt_p.lo, M, N, c->HCt_p.ld, st, c->stream));
  HIPCHK(c, split_bf16_t(SC, c->SCt_p.hi, c->SCt_p.lo, M, N, c->SCt_p.ld, st, c->stream));
  return OMM_OK;
}

// Complex problems on the real embedding: C = E(C_c) has row pairs [Re c, Im c], [-Im c, Re c],
// and so does every product whose rows follow C's (E(X) E(Y) = E(X Y), E(X)^T = E(X^H)). Such a
// product is computed for its first Mc rows and the other Mc filled by the pair rotation. Not
// in the Cholesky flavour: the real Cholesky factor of E(S) is not an embedding, so C~ = C L has
// no row pairs. Returns Mc, or 0 when every row is computed.
int paired_rows(omm_ctx* c) { return c->cplx && !reduced(c) ? (int)c->Mc : 0; }

// The second half of the rows of a paired product X (rows x cols, row length ld; type FP64 or
// FP32) and of its optional planes.
int fill_pairs(omm_ctx* c, void* X, int type, int64_t ld, int64_t cols, const Plane* p,
               bool check_done = true) {
  const int rh = paired_rows(c);
  if (!rh) return OMM_OK;
  HIPCHK(c, pair_rows(X, type == T_F64, ld, p ? p->hi : nullptr, p ? p->lo : nullptr,
                      p ? p->ld : 0, rh, (int)(cols / 2), check_done ? c->st : nullptr,
                      c->stream));
  return OMM_OK;
}

// Initial products of a phase (Sec. 2.1, Eqs. 5-6; Sec. 2.3 footnote):
//   [HC | SC] = C [Hs | S], HW = HC C^T, SW = SC C^T, E_0.
// Hs, S are symmetric, so both products read k-contiguous rows (KC x KC).
template <typename T>
int initial_products(omm_ctx* c, Work<T>& w, int compute, const T* Hs, const T* S, double* trace) {
  const int M = (int)c->M, N = (int)c->N;
  const int64_t mn = (int64_t)M * N;
  const bool bf = compute == CBF16X3;
  const int et = bf ? T_BF16P : elem_type<T>();
  if (bf) {
    TRY(alloc_iter_planes(c));
    TRY(split(c, w.C, c->C_p, M, N, false));
  }
  const Opnd Cop = bf ? pl(c->C_p) : dn(w.C, N);
  const int Mo = paired_rows(c) ? paired_rows(c) : M;  // rows computed by each product
  GemmDesc d{compute, et, et, elem_type<T>(), elem_type<T>(), KC, KC, 0, 1};
  GemmOp ops[2] = {make_op2(Mo, N, N, Cop, bf ? pl(c->Hs_p) : dn(Hs, N), w.HC, N),
                   make_op2(Mo, N, N, Cop, bf ? pl(c->S_p) : dn(S, N), w.SC, N)};
  if (sparse_products(c))  // C [Hs | S] over the non-zero K blocks only (same result)
    for (int i = 0; i < 2; ++i) {
      ops[i].kptr = c->kl_ptr[i];
      ops[i].kidx = c->kl_idx[i];
    }
  // reduced problem (S~ = I): SC = C, kept as its own copy, which every update then moves
  // exactly like C
  const bool sid = reduced(c);
  TRY(gemm(c, d, ops, sid ? 1 : 2, nullptr));
  TRY(fill_pairs(c, w.HC, elem_type<T>(), N, N, nullptr, false));
  if (!sid) TRY(fill_pairs(c, w.SC, elem_type<T>(), N, N, nullptr, false));
  if (sid)
    HIPCHK(c, hipMemcpyAsync(w.SC, w.C, mn * sizeof(T), hipMemcpyDeviceToDevice, c->stream));
  if (bf) TRY(split_state(c, w.HC, w.SC, false));
  GemmDesc d2{compute, et, et, T_F64, T_F64, KC, KC, 0, 1};
  GemmOp ops2[2] = {make_op2(Mo, M, N, bf ? pl(c->HC_p) : dn(w.HC, N), Cop, c->HW, M),
                    make_op2(Mo, M, N, bf ? pl(c->SC_p) : dn(w.SC, N), Cop, c->SW, M)};
  TRY(gemm(c, d2, ops2, 2, nullptr));
  TRY(fill_pairs(c, c->HW, T_F64, M, M, nullptr, false));
  TRY(fill_pairs(c, c->SW, T_F64, M, M, nullptr, false));
  HIPCHK(c, energy_init(c->HW, c->SW, M, c->partials, c->st, trace, c->stream));
  return OMM_OK;
}

// Event marks for profiling: 8 per line search (before stage 0 and after each stage).
int prof_mark(omm_ctx* c) {
  if (!c->prof) return OMM_OK;
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    HIPCHK(c, hipEventCreate(&e));
    c->ev_pool.push_back(e);
  }
  HIPCHK(c, hipEventRecord(c->ev_pool[c->ev_used++], c->stream));
  return OMM_OK;
}

// Fold recorded marks into per-stage milliseconds (synchronizes the stream).
int prof_collect(omm_ctx* c) {
  if (!c->prof || c->ev_used == 0) return OMM_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const size_t per = NSTAGE + 1;
  for (size_t b = 0; b + per <= c->ev_used; b += per) {
    for (int st = 0; st < NSTAGE; ++st) {
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[b + st], c->ev_pool[b + st + 1]));
      c->stage_ms[st] += ms;
    }
    c->prof_iters += 1;
  }
  c->ev_used = 0;
  return OMM_OK;
}

bool fuse_enabled() {
  const char* e = getenv("OMM_FUSE");
  return !(e && e[0] == '0');
}

bool pg_split_enabled() {
  const char* e = getenv("OMM_PG_SPLIT");
  return e && e[0] == '1';
}

// One line search (the stage sequence in the header comment of this file). In BF16x3 mode every
// GEMM operand is split into bf16 hi/lo planes once, right after it is produced.
template <typename T>
int line_search_iteration(omm_ctx* c, Work<T>& w, int compute, const T* Hs, const T* S,
                          const T* P, int k, double* trace) {
  const int M = (int)c->M, N = (int)c->N;
  const int64_t mn = (int64_t)M * N;
  const bool bf = compute == CBF16X3;
  // BF16: the operand planes of G, HD, SD come from the GEMM epilogues and those of HC, SC from
  // the update kernel; OMM_FUSE=0 splits them in separate passes instead (same values)
  const bool fuse = bf && fuse_enabled();
  const int Mo = paired_rows(c) ? paired_rows(c) : M;  // rows computed by each product
  const int et = elem_type<T>();
  const int ot = bf ? T_BF16P : et;  // operand element type of the GEMMs
  const int* done = &c->st->done;
  // BF16 with the FP64 state: the products G, PG, HD, SD are stored in FP32 (see Work)
  const bool f32p = bf && sizeof(T) == 8 && w.PGf != nullptr;
  T* G = (k & 1) ? w.Gp : w.G;
  T* Gprev = (k & 1) ? w.G : w.Gp;
  float* Gf = (k & 1) ? w.Gpf : w.Gf;
  float* Gfprev = (k & 1) ? w.Gf : w.Gpf;
  void* Gout = f32p ? (void*)Gf : (void*)G;
  const int tg = f32p ? T_F32 : et;
  TRY(prof_mark(c));
  // G = 8 HC - 4 HW SC - 4 SW HC
  {
    if (bf) {
      TRY(split(c, c->HW, c->HW_p, M, M));
      TRY(split(c, c->SW, c->SW_p, M, M));
    }
    // BF16x3 reads the transposed planes of SC, HC (k-contiguous); the others read SC, HC by rows
    GemmDesc d{compute, bf ? T_BF16P : T_F64, ot, tg, et, KC, bf ? KC : RC, 0, 1};
    GemmOp op = make_op2(Mo, N, M, bf ? pl(c->HW_p) : dn(c->HW, M),
                         bf ? pl(c->SCt_p) : dn(w.SC, N), Gout, N, -4.0, w.HC, N, 8.0);
    const Opnd a2 = bf ? pl(c->SW_p) : dn(c->SW, M), b2 = bf ? pl(c->HCt_p) : dn(w.HC, N);
    op.nseg = 2;
    op.A[1] = a2.p; op.Alo[1] = a2.lo; op.lda[1] = a2.ld;
    op.B[1] = b2.p; op.Blo[1] = b2.lo; op.ldb[1] = b2.ld;
    op.K[1] = M;
    // G's bf16 plane for the preconditioner product, from the epilogue (the product takes G
    // rounded to bf16: no lo plane, unless OMM_PG_SPLIT=1)
    if (fuse && c->p_kind > 0) {
      out_planes(op, c->G_p);
      if (!pg_split_enabled()) op.Clo = nullptr;
    }
    TRY(gemm(c, d, &op, 1, done));
    TRY(fill_pairs(c, Gout, tg, N, N, fuse && c->p_kind > 0 ? &c->G_p : nullptr));
  }
  TRY(prof_mark(c));
  // BF16x3: the preconditioner is applied as its bf16 rounding P~ (the hi plane of P, a symmetric
  // matrix of its own) to the bf16 rounding G~ of G, a single MFMA product, and the search
  // direction is rounded to bf16 when it is formed, so every product with D takes two MFMA
  // products instead of three (same accuracy: the rounded operand is exact). PG only shapes the
  // search direction; the line search is exact along whatever D results. Each element of G~ is
  // within 2^-9 of G's, but PG = G~ P~ sums N terms: its error is bounded by ~2^-9 |G| |P|
  // per element, not relative to PG, which can be much smaller under cancellation, and the
  // rounding of G makes the applied preconditioner vary from one line search to the next.
  // OMM_PG_SPLIT=1 applies P~ to G's hi/lo planes instead (two MFMA products, G exact to
  // ~2^-17).
  const bool pg_split = bf && pg_split_enabled();
  const int cP = bf ? (pg_split ? CBF16X2B : CBF16X1) : compute, cD = bf ? CBF16X2A : compute;
  T* PG = G;
  if (c->p_kind > 0) {
    if (bf && !fuse) {
      if (f32p) TRY(split(c, Gf, c->G_p, M, N));
      else TRY(split(c, G, c->G_p, M, N));
    }
    const int tp = f32p ? T_F32 : et;
    GemmDesc d{cP, ot, ot, tp, tp, KC, KC, 0, 1};
    GemmOp op = make_op2(Mo, N, N, bf ? pl(c->G_p) : dn(G, N), bf ? pl(c->P_p) : dn(P, N),
                         f32p ? (void*)w.PGf : (void*)w.PG, N);
    TRY(gemm(c, d, &op, 1, done));
    TRY(fill_pairs(c, f32p ? (void*)w.PGf : (void*)w.PG, tp, N, N, nullptr));
    PG = w.PG;
  }
  TRY(prof_mark(c));
  // BF16: D lives in its bf16 plane (exact); the fused update reads it there, so the T copy is
  // written only for the separate update
  T* Dcopy = fuse ? nullptr : w.D;
  if (f32p && c->p_kind > 0)
    HIPCHK(c, (beta_and_direction<T, float, float>(Gf, w.PGf, Gfprev, Dcopy, mn, k == 0 ? 1 : 0,
                                                  c->partials, c->st, c->stream, c->D_p.hi, N,
                                                  c->D_p.ld)));
  else if (f32p)  // no preconditioner: PG = G
    HIPCHK(c, (beta_and_direction<T, float, float>(Gf, Gf, Gfprev, Dcopy, mn, k == 0 ? 1 : 0,
                                                  c->partials, c->st, c->stream, c->D_p.hi, N,
                                                  c->D_p.ld)));
  else
    HIPCHK(c, beta_and_direction<T>(G, PG, Gprev, Dcopy, mn, k == 0 ? 1 : 0, c->partials, c->st,
                                    c->stream, bf ? c->D_p.hi : nullptr, N, c->D_p.ld));
  TRY(prof_mark(c));
  const Opnd Dop = bf ? pl(c->D_p) : dn(w.D, N);
  // reduced problem (S~ = I): SD = D, no product
  const bool sid = reduced(c);
  T* SD = sid ? w.D : w.SD;
  const bool hdf = f32p && !sid;  // with S~ = I, SD is D itself (FP64)
  {
    const int td = hdf ? T_F32 : et;
    GemmDesc d{cD, ot, ot, td, td, KC, KC, 0, 1};
    GemmOp ops[2] = {make_op2(Mo, N, N, Dop, bf ? pl(c->Hs_p) : dn(Hs, N),
                              hdf ? (void*)w.HDf : (void*)w.HD, N),
                     make_op2(Mo, N, N, Dop, bf ? pl(c->S_p) : dn(S, N),
                              hdf ? (void*)w.SDf : (void*)w.SD, N)};
    if (bf && sparse_products(c)) {
      for (int i = 0; i < 2; ++i) {
        ops[i].kptr = c->kl_ptr[i];
        ops[i].kidx = c->kl_idx[i];
      }
    }
    if (fuse) {  // the projection stage's operand planes, from the epilogue
      out_planes(ops[0], c->HD_p);
      out_planes(ops[1], c->SD_p);
    }
    TRY(gemm(c, d, ops, sid ? 1 : 2, done));
    TRY(fill_pairs(c, ops[0].C, td, N, N, fuse ? &c->HD_p : nullptr));
    if (!sid) TRY(fill_pairs(c, ops[1].C, td, N, N, fuse ? &c->SD_p : nullptr));
  }
  TRY(prof_mark(c));
  if (bf && !fuse) {  // the projection stage's operand planes (D's lo plane stays zero)
    if (hdf) {
      TRY(split(c, w.HDf, c->HD_p, M, N));
      TRY(split(c, w.SDf, c->SD_p, M, N));
    } else {
      TRY(split(c, w.HD, c->HD_p, M, N));
      if (!sid) TRY(split(c, w.SD, c->SD_p, M, N));
    }
  }
  const Plane& SD_p = sid ? c->D_p : c->SD_p;
  {
    GemmDesc d{cD, ot, ot, T_F64, T_F64, KC, KC, 0, 1};
    GemmOp ops[4] = {make_op2(Mo, M, N, Dop, bf ? pl(c->HC_p) : dn(w.HC, N), c->H1, M),
                     make_op2(Mo, M, N, Dop, bf ? pl(c->SC_p) : dn(w.SC, N), c->S1, M),
                     make_op2(Mo, M, N, Dop, bf ? pl(c->HD_p) : dn(w.HD, N), c->H2, M),
                     make_op2(Mo, M, N, Dop, bf ? pl(SD_p) : dn(SD, N), c->S2, M)};
    // H'' = D Hs D^T and S'' = D S D^T are symmetric (Eq. 15): their upper block triangles are
    // computed and mirrored (square products only: not with paired rows)
    if (Mo == M) ops[2].tri = ops[3].tri = 1;
    TRY(gemm(c, d, ops, 4, done));
    for (double* X : {c->H1, c->S1, c->H2, c->S2}) TRY(fill_pairs(c, X, T_F64, M, M, nullptr));
  }
  TRY(prof_mark(c));
  HIPCHK(c, line_search(c->HW, c->SW, c->H1, c->S1, c->H2, c->S2, M, c->partials, c->st,
                        c->stream));
  TRY(prof_mark(c));
  if (fuse) {  // with the planes of the new HC, SC and of their transposes
    const StatePlanes sp{c->HC_p.hi,  c->HC_p.lo,  c->SC_p.hi,  c->SC_p.lo,
                         c->HCt_p.hi, c->HCt_p.lo, c->SCt_p.hi, c->SCt_p.lo,
                         c->HC_p.ld,  c->HCt_p.ld};
    if (hdf)
      HIPCHK(c, (update_coefficients_split<T, float>(w.C, c->D_p.hi, c->D_p.ld, w.HC, w.HDf, w.SC,
                                                    w.SDf, M, N, sp, c->st, c->stream)));
    else
      HIPCHK(c, update_coefficients_split<T>(w.C, c->D_p.hi, c->D_p.ld, w.HC, w.HD, w.SC,
                                             sid ? nullptr : w.SD, M, N, sp, c->st, c->stream));
  } else {
    if (hdf)
      HIPCHK(c, (update_coefficients<T, float>(w.C, w.D, w.HC, w.HDf, w.SC, w.SDf, mn, c->st,
                                              c->stream)));
    else
      HIPCHK(c, update_coefficients<T>(w.C, w.D, w.HC, w.HD, w.SC, SD, mn, c->st, c->stream));
    if (bf) TRY(split_state(c, w.HC, w.SC));
  }
  HIPCHK(c, update_subspace(c->HW, c->SW, c->H1, c->S1, c->H2, c->S2, M, c->partials, c->st,
                            trace, c->stream));
  TRY(prof_mark(c));
  return OMM_OK;
}

int read_state(omm_ctx* c) {
  HIPCHK(c, hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return OMM_OK;
}

int ensure_trace(omm_ctx* c, int need) {
  if (c->trace_cap >= need) return OMM_OK;
  double* t = nullptr;
  TRY(dalloc(c, &t, (size_t)need));
  if (c->trace) {
    HIPCHK(c, hipMemcpyAsync(t, c->trace, c->trace_cap * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graph(c);  // a captured graph holds the old trace address
    dfree(c->trace);
  }
  c->trace = t;
  c->trace_cap = need;
  return OMM_OK;
}

void drop_graph(omm_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
  c->graph_parity = -1;
}

bool graphs_enabled(omm_ctx* c) {
  const char* e = getenv("OMM_GRAPH");
  return !c->prof && !(e && e[0] == '0');
}

// Captures line searches k and k+1 (same buffers every time; only the parity of k matters).
template <typename T>
int capture_pair(omm_ctx* c, Work<T>& w, int compute, const T* Hs, const T* S, const T* P, int k,
                 double* trace) {
  drop_graph(c);
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  int r = line_search_iteration<T>(c, w, compute, Hs, S, P, k, trace);
  if (r == OMM_OK) r = line_search_iteration<T>(c, w, compute, Hs, S, P, k + 1, trace);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (r != OMM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  HIPCHK(c, e);
  c->graph = g;
  HIPCHK(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
  c->graph_parity = k & 1;
  return OMM_OK;
}

// Starts a CG phase in precision T: initial products and E_0 (the state's iteration count 0).
template <typename T>
int phase_begin(omm_ctx* c, Work<T>& w, int compute, const T* Hs, const T* S, double tol,
                int trace_off) {
  DevState init{};
  init.tol = tol;
  init.max_iter = 0;
  HIPCHK(c, hipMemcpyAsync(c->st, &init, sizeof(DevState), hipMemcpyHostToDevice, c->stream));
  TRY(ensure_trace(c, trace_off + 2));
  drop_graph(c);
  TRY(initial_products<T>(c, w, compute, Hs, S, c->trace + trace_off));
  TRY(read_state(c));
  c->phase_active = true;
  c->phase_k = 0;
  c->trace_off = trace_off;
  return OMM_OK;
}

// Up to `count` more line searches of the active phase (stops early on convergence / error).
template <typename T>
int phase_iterate(omm_ctx* c, Work<T>& w, int compute, const T* Hs, const T* S, const T* P,
                  double tol, int count, int* done_out) {
  DevState* h = c->st_host;
  if (h->done < 0) {
    *done_out = h->done;
    return OMM_OK;
  }
  h->done = 0;
  h->tol = tol;
  h->max_iter = h->iter + count;
  TRY(ensure_trace(c, c->trace_off + h->max_iter + 2));
  HIPCHK(c, hipMemcpyAsync(c->st, h, sizeof(DevState), hipMemcpyHostToDevice, c->stream));
  double* trace = c->trace + c->trace_off;
  // Host checks the device state every `check` launches; iterations launched after the stop
  // return immediately.
  const int check = c->N >= 4096 ? 2 : 8;
  if (count > 0) {
    // The first two line searches of a phase run eagerly (every GEMM shape is tuned and its
    // workspace allocated); after that pairs of line searches replay one captured graph.
    const bool graphs = graphs_enabled(c);
    int since = 0;
    for (int k = 0; k < count;) {
      if (graphs && c->phase_k >= 2 && count - k >= 2) {
        if (!c->graph_exec || c->graph_parity != (c->phase_k & 1))
          TRY(capture_pair<T>(c, w, compute, Hs, S, P, c->phase_k, trace));
        HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
        k += 2;
        c->phase_k += 2;
        since += 2;
      } else {
        TRY(line_search_iteration<T>(c, w, compute, Hs, S, P, c->phase_k, trace));
        k += 1;
        c->phase_k += 1;
        since += 1;
      }
      if (since >= check || k == count) {
        since = 0;
        TRY(read_state(c));
        if (h->done != 0) break;
      }
    }
    TRY(prof_collect(c));
  }
  TRY(read_state(c));
  *done_out = count > 0 ? h->done : 2;
  if (*done_out == 0) *done_out = 2;
  return OMM_OK;
}

// FP64 resynchronization of the CG state from C (Sec. 2.1, Eqs. 5-6): HC, SC, HW, SW and the
// energy are recomputed exactly, removing what the BF16x3 increments accumulated.
int resync_fp64(omm_ctx* c) {
  const int M = (int)c->M, N = (int)c->N;
  Work<double>& w = c->w64;
  GemmDesc d{CF64, T_F64, T_F64, T_F64, T_F64, KC, KC, 0, 1};
  const bool sid = reduced(c);
  const int Mo = paired_rows(c) ? paired_rows(c) : M;  // rows computed by each product
  GemmOp ops[2] = {make_op(Mo, N, N, w.C, N, c->Hs, N, w.HC, N),
                   make_op(Mo, N, N, w.C, N, c->S, N, w.SC, N)};
  if (sparse_products(c))  // the FP64 products skip the same zero blocks of Hs and S
    for (int i = 0; i < 2; ++i) {
      ops[i].kptr = c->kl_ptr[i];
      ops[i].kidx = c->kl_idx[i];
    }
  TRY(gemm(c, d, ops, sid ? 1 : 2, nullptr));
  TRY(fill_pairs(c, w.HC, T_F64, N, N, nullptr, false));
  if (!sid) TRY(fill_pairs(c, w.SC, T_F64, N, N, nullptr, false));
  if (sid)
    HIPCHK(c, hipMemcpyAsync(w.SC, w.C, (size_t)M * N * sizeof(double), hipMemcpyDeviceToDevice,
                             c->stream));
  GemmOp ops2[2] = {make_op(Mo, M, N, w.HC, N, w.C, N, c->HW, M),
                    make_op(Mo, M, N, w.SC, N, w.C, N, c->SW, M)};
  TRY(gemm(c, d, ops2, 2, nullptr));
  TRY(fill_pairs(c, c->HW, T_F64, M, M, nullptr, false));
  TRY(fill_pairs(c, c->SW, T_F64, M, M, nullptr, false));
  // the BF16x3 products read HC and SC through their planes
  TRY(split_state(c, w.HC, w.SC, false));
  const int it = c->st_host->iter;
  TRY(ensure_trace(c, c->trace_off + it + 2));
  HIPCHK(c, energy_init(c->HW, c->SW, M, c->partials, c->st, c->trace + c->trace_off + it,
                        c->stream));
  TRY(read_state(c));
  c->since_resync = 0;
  c->ck_iter.push_back(it);
  c->ck_E.push_back(c->st_host->E);
  return OMM_OK;
}

// Up to `count` line searches of the mixed scheme: BF16x3 products, FP64 state, an FP64
// resynchronization every `resync_every` line searches. The stopping rule (Eq. 18) is applied
// to consecutive FP64-exact energies, scaled by the number of line searches between them. The
// schedule counts line searches since the last resynchronization across calls; `close` adds
// one at the end of the call when the last line search did not fall on the schedule.
int mixed64_iterate(omm_ctx* c, double tol, int count, bool close, int* done_out) {
  const int K = c->resync_every > 0 ? c->resync_every : 20;
  const double* P = c->p_kind > 0 ? c->P : nullptr;
  int left = count;
  *done_out = 2;
  while (left > 0) {
    const int n = std::min(left, K - c->since_resync);
    int d = 0;
    TRY(phase_iterate<double>(c, c->w64, CBF16X3, c->Hs, c->S, P, 0.0, n, &d));
    left -= n;
    c->since_resync += n;
    if (d < 0) {
      *done_out = d;
      return OMM_OK;
    }
    if (c->since_resync >= K || (left == 0 && close)) {
      const int span = c->since_resync;
      const double E_old = c->resync_E;
      TRY(resync_fp64(c));
      const double E = c->st_host->E;
      c->resync_E = E;
      if (!std::isfinite(E)) {
        *done_out = -5;
        return OMM_OK;
      }
      if (fabs(2.0 * (E - E_old)) <= span * tol * fabs(E + E_old)) {
        *done_out = 1;
        return OMM_OK;
      }
    }
  }
  return OMM_OK;
}

int status_of_done(omm_ctx* c, int done) {
  switch (done) {
    case 1: return OMM_OK;
    case 2: return fail(c, OMM_W_MAXITER, "max_iter line searches without meeting tol");
    case -5: return fail(c, OMM_E_NONFINITE, "non-finite value in the iteration");
    case -7:
      return fail(c, OMM_E_NO_LINE_MIN,
                  "the quartic along the search direction has no local minimum (is eta above "
                  "the M-th eigenvalue?)");
    case -8: return fail(c, OMM_E_DIVERGED, "Tr SW exceeded 16 M: the iteration diverged");
    default: return fail(c, OMM_E_HIP, "unexpected device state");
  }
}

int minimize_impl(omm_ctx* c, const double* C0, bool C0_device, double eta, double tau, double tol,
                  int max_iter) {
  if (!c) return OMM_E_ARG;
  if (!c->have_HS) return fail(c, OMM_E_STATE, "omm_set_HS must be called before omm_minimize");
  if (!(tol >= 0.0) || max_iter < 0 || !std::isfinite(eta) || std::isnan(tau))
    return fail(c, OMM_E_ARG, "need tol >= 0, max_iter >= 0, finite eta, non-NaN tau");
  if (!C0 && !c->have_C) return fail(c, OMM_E_STATE, "no C0 given and no C to resume from");
  if (!C0 && c->c_flavour != c->flavour)
    return fail(c, OMM_E_STATE, "the flavour changed since the last minimization: pass C0");
  const size_t mn = (size_t)c->M * c->N;
  TRY(alloc_common(c));
  TRY(alloc_work<double>(c, c->w64));
  const bool mixed64 = c->mode == OMM_BF16X3 && c->refine;
  if (c->mode != OMM_FP64 && !mixed64) TRY(alloc_work<float>(c, c->w32));
  TRY(prepare_shift(c, eta));
  TRY(prepare_precon(c, tau));
  c->eta_last = eta;

  // Load C into the working precision of phase 1.
  if (C0) {
    if (C0_device) HIPCHK(c, hipMemcpyAsync(c->w64.C, C0, mn * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    else HIPCHK(c, hipMemcpyAsync(c->w64.C, C0, mn * sizeof(double), hipMemcpyHostToDevice, c->stream));
    c->c_prec = OMM_FP64;
    if (reduced(c)) {  // C~0 = C0 L: B(n, k) = L[k][n] (RC)
      const int M = (int)c->M, N = (int)c->N;
      GemmDesc d{CF64, T_F64, T_F64, T_F64, T_F64, KC, RC, 0, 1};
      GemmOp op = make_op(M, N, N, c->w64.C, N, c->L, N, c->w64.HD, N);
      TRY(gemm(c, d, &op, 1, nullptr));
      HIPCHK(c, hipMemcpyAsync(c->w64.C, c->w64.HD, mn * sizeof(double), hipMemcpyDeviceToDevice,
                               c->stream));
    }
    c->c_flavour = c->flavour;
  }
  if (c->mode != OMM_FP64 && !mixed64 && c->c_prec == OMM_FP64)
    HIPCHK(c, convert_f64_f32(c->w64.C, c->w32.C, (int64_t)mn, c->stream));
  if ((c->mode == OMM_FP64 || mixed64) && c->c_prec != OMM_FP64)
    HIPCHK(c, convert_f32_f64(c->w32.C, c->w64.C, (int64_t)mn, c->stream));
  c->have_C = true;

  int done1 = 0, done2 = 0;
  c->iters = 0;
  c->iters_before = 0;
  c->phase_mixed64 = false;
  c->ck_iter.clear();
  c->ck_E.clear();
  if (mixed64) {
    TRY(phase_begin<double>(c, c->w64, CF64, c->Hs, c->S, tol, 0));
    TRY(alloc_iter_planes(c));
    TRY(split_state(c, c->w64.HC, c->w64.SC, false));
    c->phase_prec = OMM_BF16X3;
    c->phase_mixed64 = true;
    c->since_resync = 0;
    c->resync_E = c->st_host->E;
    c->ck_iter.push_back(0);
    c->ck_E.push_back(c->st_host->E);
    TRY(mixed64_iterate(c, tol, max_iter, true, &done1));
    c->c_prec = OMM_FP64;
    c->iters = c->st_host->iter;
    c->trace_n = c->iters + 1;
  } else if (c->mode == OMM_FP64) {
    TRY(phase_begin<double>(c, c->w64, CF64, c->Hs, c->S, tol, 0));
    c->phase_prec = OMM_FP64;
    TRY(phase_iterate<double>(c, c->w64, CF64, c->Hs, c->S, c->p_kind > 0 ? c->P : nullptr, tol,
                              max_iter, &done1));
    c->c_prec = OMM_FP64;
    c->iters = c->st_host->iter;
    c->trace_n = c->iters + 1;
  } else {
    const int comp = compute_of(c->mode);
    const double tol1 = c->refine ? fmax(tol, c->mixed_tol) : tol;
    TRY(phase_begin<float>(c, c->w32, comp, c->Hs32, c->S32, tol1, 0));
    c->phase_prec = c->mode;
    TRY(phase_iterate<float>(c, c->w32, comp, c->Hs32, c->S32, c->p_kind > 0 ? c->P32 : nullptr,
                             tol1, max_iter, &done1));
    c->c_prec = c->mode;
    const int iters1 = c->st_host->iter;
    c->iters = iters1;
    c->trace_n = iters1 + 1;
    if (done1 < 0) return status_of_done(c, done1);
    if (c->refine) {
      HIPCHK(c, convert_f32_f64(c->w32.C, c->w64.C, (int64_t)mn, c->stream));
      c->c_prec = OMM_FP64;
      c->iters_before = iters1;
      TRY(phase_begin<double>(c, c->w64, CF64, c->Hs, c->S, tol, iters1 + 1));
      c->phase_prec = OMM_FP64;
      TRY(phase_iterate<double>(c, c->w64, CF64, c->Hs, c->S, c->p_kind > 0 ? c->P : nullptr,
                                tol, max_iter, &done2));
      c->iters = iters1 + c->st_host->iter;
      c->trace_n = iters1 + 1 + c->st_host->iter + 1;
      done1 = done2;
    }
  }
  c->last_rel = c->st_host->rel_change;
  c->trace_host.assign((size_t)c->trace_n, 0.0);
  HIPCHK(c, hipMemcpyAsync(c->trace_host.data(), c->trace, c->trace_n * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return status_of_done(c, done1);
}

// C in FP64 (converting from the mixed-precision working copy if that is where it lives).
int c64(omm_ctx* c) {
  if (!c->have_C) return fail(c, OMM_E_STATE, "no minimization has run");
  if (c->c_prec != OMM_FP64) {
    HIPCHK(c, convert_f32_f64(c->w32.C, c->w64.C, (int64_t)c->M * c->N, c->stream));
    c->c_prec = OMM_FP64;
  }
  return OMM_OK;
}

// C in the original basis (FP64): the working C, or C = C~ L^-1 in the reduced flavour.
int c_original(omm_ctx* c, const double** out) {
  TRY(c64(c));
  if (c->c_flavour != OMM_FLAVOUR_CHOLESKY) {
    *out = c->w64.C;
    return OMM_OK;
  }
  if (!c->l_valid) return fail(c, OMM_E_STATE, "the Cholesky factor is gone (new S): minimize again");
  const int M = (int)c->M, N = (int)c->N;
  TRY(dalloc(c, &c->Corig, (size_t)M * N));
  GemmDesc d{CF64, T_F64, T_F64, T_F64, T_F64, KC, RC, 0, 1};  // B(n, k) = L^-1[k][n]
  GemmOp op = make_op(M, N, N, c->w64.C, N, c->Linv, N, c->Corig, N);
  TRY(gemm(c, d, &op, 1, nullptr));
  *out = c->Corig;
  return OMM_OK;
}

// out = scale * C^T X C-style products: rho = 2 C^T (2I - SW) C, EDM = 2 C^T HW C.
int ct_x_c(omm_ctx* c, const double* Xmm, double diag_for_identity, bool use_identity,
           double* out) {
  const double* Cb = nullptr;
  TRY(c_original(c, &Cb));
  const int M = (int)c->M, N = (int)c->N;
  double* Y = c->H1;  // M x M scratch
  if (use_identity) HIPCHK(c, identity_minus(Xmm, Y, M, diag_for_identity, 1.0, c->stream));
  else HIPCHK(c, copy_f64(Xmm, Y, (int64_t)M * M, c->stream));
  double* Z = c->w64.HD;  // M x N scratch: Z = Y C
  GemmDesc d{CF64, T_F64, T_F64, T_F64, T_F64, KC, RC, 0, 1};
  GemmOp op = make_op(M, N, M, Y, M, Cb, N, Z, N);
  TRY(gemm(c, d, &op, 1, nullptr));
  // out = 2 C^T Z : A(m, k) = C[k, m] (RC), B(k, n) = Z[k, n] (RC)
  GemmDesc d2{CF64, T_F64, T_F64, T_F64, T_F64, RC, RC, 0, 1};
  GemmOp op2 = make_op(N, N, M, Cb, N, Z, N, out, N, 2.0);
  TRY(gemm(c, d2, &op2, 1, nullptr));
  return OMM_OK;
}

int need_minimized(omm_ctx* c) {
  if (!c->have_C || !c->HW) return fail(c, OMM_E_STATE, "no minimization has run");
  return OMM_OK;
}

}  // namespace

// [[A, B], [-B, A]] (2n x 2n) from the real and imaginary parts (n x n; im nullable = 0).
void omm::embed_operator(const double* re, const double* im, int64_t n, std::vector<double>& out) {
  const int64_t n2 = 2 * n;
  out.assign((size_t)n2 * n2, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      const double a = re[i * n + j], b = im ? im[i * n + j] : 0.0;
      out[i * n2 + j] = a;
      out[(i + n) * n2 + j + n] = a;
      out[i * n2 + j + n] = b;
      out[(i + n) * n2 + j] = -b;
    }
}

// Rows [Re c_i, Im c_i] (i < m) and [-Im c_i, Re c_i] (2m x 2n) of the complex m x n C.
void omm::embed_rows(const double* re, const double* im, int64_t m, int64_t n, std::vector<double>& out) {
  const int64_t n2 = 2 * n;
  out.assign((size_t)(2 * m) * n2, 0.0);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) {
      const double a = re[i * n + j], b = im ? im[i * n + j] : 0.0;
      out[i * n2 + j] = a;
      out[i * n2 + j + n] = b;
      out[(i + m) * n2 + j] = -b;
      out[(i + m) * n2 + j + n] = a;
    }
}


extern "C" {

int omm_create(int64_t N, int64_t M, omm_ctx** out) {
  if (!out) return OMM_E_ARG;
  *out = nullptr;
  if (N <= 0 || M <= 0 || M > N || N > (int64_t)1 << 30) return OMM_E_ARG;
  omm_ctx* c = new omm_ctx();
  c->N = N;
  c->M = M;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return OMM_E_HIP;
  }
  if (hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return OMM_E_HIP;
  }
  c->stream = c->own;
  *out = c;
  return OMM_OK;
}

int omm_destroy(omm_ctx* c) {
  if (!c) return OMM_E_ARG;
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  dfree(c->H); dfree(c->S); dfree(c->T); dfree(c->Hs); dfree(c->P);
  dfree(c->Hs32); dfree(c->S32); dfree(c->P32);
  free_work(c->w64);
  free_work(c->w32);
  for (Plane* p : {&c->Hs_p, &c->S_p, &c->P_p, &c->C_p, &c->HC_p, &c->SC_p, &c->G_p, &c->D_p,
                   &c->HD_p, &c->SD_p, &c->HW_p, &c->SW_p, &c->HCt_p, &c->SCt_p})
    free_plane(*p);
  dfree(c->HW); dfree(c->SW); dfree(c->H1); dfree(c->S1); dfree(c->H2); dfree(c->S2);
  dfree(c->partials); dfree(c->ws); dfree(c->st); dfree(c->flags); dfree(c->trace);
  dfree(c->nn_scratch); dfree(c->inv_work);
  dfree(c->L); dfree(c->Linv); dfree(c->Corig);
  for (int i = 0; i < 2; ++i) {
    dfree(c->kl_ptr[i]);
    dfree(c->kl_idx[i]);
  }
  if (c->st_host) (void)hipHostFree(c->st_host);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->own) (void)hipStreamDestroy(c->own);
  delete c;
  return OMM_OK;
}

int omm_set_precision(omm_ctx* c, int mode, int fp64_refine) {
  if (!c) return OMM_E_ARG;
  if (mode != OMM_FP64 && mode != OMM_FP32 && mode != OMM_BF16X3)
    return fail(c, OMM_E_ARG, "unknown precision mode");
  c->mode = mode;
  c->refine = fp64_refine ? 1 : 0;
  return OMM_OK;
}

int omm_set_flavour(omm_ctx* c, int flavour) {
  if (!c) return OMM_E_ARG;
  if (flavour != OMM_FLAVOUR_DENSE && flavour != OMM_FLAVOUR_CHOLESKY)
    return fail(c, OMM_E_ARG, "unknown flavour");
  if (flavour != c->flavour) {
    drop_graph(c);
    c->flavour = flavour;
    c->phase_active = false;
    c->phase_mixed64 = false;
  }
  return OMM_OK;
}

int omm_set_sparse(omm_ctx* c, int on) {
  if (!c) return OMM_E_ARG;
  if ((on != 0) != c->sparse) {
    drop_graph(c);
    c->sparse = on != 0;
  }
  return OMM_OK;
}

int omm_sparse_density(omm_ctx* c, double* density) {
  if (!c || !density) return c ? fail(c, OMM_E_ARG, "null output") : OMM_E_ARG;
  if (!c->kl_valid[0] || !c->kl_valid[1])
    return fail(c, OMM_E_STATE, "no block-sparse lists: enable sparse products and minimize");
  density[0] = c->kl_density[0];
  density[1] = c->kl_density[1];
  return OMM_OK;
}

int omm_set_mixed_tol(omm_ctx* c, double tol) {
  if (!c) return OMM_E_ARG;
  if (!(tol >= 0.0)) return fail(c, OMM_E_ARG, "tol must be >= 0");
  c->mixed_tol = tol;
  return OMM_OK;
}

int omm_set_resync(omm_ctx* c, int every) {
  if (!c) return OMM_E_ARG;
  if (every < 1) return fail(c, OMM_E_ARG, "resync interval must be >= 1");
  c->resync_every = every;
  return OMM_OK;
}

int omm_checkpoints(omm_ctx* c, int* iters, double* energies, int cap, int* n) {
  if (!c || ((!iters || !energies) && cap > 0)) return c ? fail(c, OMM_E_ARG, "null buffer") : OMM_E_ARG;
  const int k = std::min(cap, (int)c->ck_E.size());
  for (int i = 0; i < k; ++i) {
    iters[i] = c->ck_iter[i];
    energies[i] = c->ck_E[i] * (c->cplx ? 0.5 : 1.0);
  }
  if (n) *n = (int)c->ck_E.size();
  return OMM_OK;
}

int omm_set_stream(omm_ctx* c, void* s) {
  if (!c) return OMM_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->stream = s ? (hipStream_t)s : c->own;
  return OMM_OK;
}

// Copies the symmetrized S and T in from `src_S`, `src_T` (device, or host through the Hs
// buffer as staging: Hs is rebuilt from H and S before it is read again) and reports whether
// either changed bit for bit; with no earlier S and T (or T added or dropped) they count as
// changed.
int load_S_T(omm_ctx* c, const double* src_S, const double* src_T, bool host, bool* changed) {
  const int64_t n = c->N;
  const size_t nn = (size_t)n * n, bytes = nn * sizeof(double);
  const bool compare = c->have_HS && (src_T != nullptr) == c->have_T;
  c->have_HS = false;  // until the new inputs are all in
  if (src_T) TRY(dalloc(c, &c->T, nn));
  TRY(dalloc(c, &c->flags, 8));
  TRY(dalloc(c, &c->Hs, nn));
  c->hs_valid = false;
  int diff = compare ? 0 : 1;
  HIPCHK(c, hipMemcpyAsync(c->flags + 2, &diff, sizeof(int), hipMemcpyHostToDevice, c->stream));
  double* dsts[2] = {c->S, c->T};
  const double* srcs[2] = {src_S, src_T};
  for (int k = 0; k < 2; ++k) {
    if (!srcs[k]) continue;
    // staged and symmetrized first, so that the stored copy is compared with what would be stored
    HIPCHK(c, hipMemcpyAsync(c->Hs, srcs[k], bytes,
                             host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, symmetrize(c->Hs, n, c->stream));
    HIPCHK(c, copy_compare_f64(c->Hs, dsts[k], (int64_t)nn, c->flags + 2, c->stream));
  }
  HIPCHK(c, hipMemcpyAsync(&diff, c->flags + 2, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *changed = diff != 0;
  return OMM_OK;
}

// S and T (compared with the stored copies), then H, from host or device memory. On failure the
// inputs count as absent and everything derived from them is dropped.
int load_inputs(omm_ctx* c, const double* H, const double* S, const double* T, bool host) {
  const size_t bytes = (size_t)c->N * c->N * sizeof(double);
  bool st_changed = true;
  int r = load_S_T(c, S, T, host, &st_changed);
  if (r == OMM_OK) {
    const hipError_t e0 = hipMemcpyAsync(c->H, H, bytes,
                                         host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                                         c->stream);
    const hipError_t e1 = e0 == hipSuccess ? symmetrize(c->H, c->N, c->stream) : e0;
    const hipError_t e2 = e1 == hipSuccess ? hipStreamSynchronize(c->stream) : e1;
    if (e2 != hipSuccess) r = fail(c, OMM_E_HIP, std::string("copying H: ") + hipGetErrorString(e2));
  }
  if (r != OMM_OK) {
    invalidate(c, true);
    return r;
  }
  c->have_T = T != nullptr;
  c->have_HS = true;
  invalidate(c, st_changed);
  return OMM_OK;
}

int omm_set_HS(omm_ctx* c, const double* H, const double* S, const double* T) {
  if (!c) return OMM_E_ARG;
  if (!H || !S) return fail(c, OMM_E_ARG, "H and S are required");
  const int64_t n = c->N;
  const double* mats[3] = {H, S, T};
  const char* names[3] = {"H", "S", "T"};
  for (int i = 0; i < 3; ++i) {
    if (!mats[i]) continue;
    bool fin = true;
    if (!host_check(mats[i], n, &fin)) {
      if (!fin) return fail(c, OMM_E_NONFINITE, std::string(names[i]) + " has a non-finite entry");
      return fail(c, OMM_E_ASYMMETRIC, std::string(names[i]) + " is not symmetric");
    }
  }
  TRY(ensure_inputs(c));
  // Validated to 1e-10; store exactly symmetric copies so that every operator product may read
  // rows in place of columns.
  return load_inputs(c, H, S, T, true);
}

int omm_set_HS_device(omm_ctx* c, const double* dH, const double* dS, const double* dT) {
  if (!c) return OMM_E_ARG;
  if (!dH || !dS) return fail(c, OMM_E_ARG, "H and S are required");
  const int64_t n = c->N;
  TRY(ensure_inputs(c));
  TRY(dalloc(c, &c->flags, 8));
  const double* mats[3] = {dH, dS, dT};
  const char* names[3] = {"H", "S", "T"};
  for (int i = 0; i < 3; ++i) {
    if (!mats[i]) continue;
    int h[2] = {0, 0};
    HIPCHK(c, hipMemsetAsync(c->flags, 0, 2 * sizeof(int), c->stream));
    HIPCHK(c, validate_symmetric(mats[i], n, 1e-10, c->flags, c->stream));
    HIPCHK(c, hipMemcpyAsync(h, c->flags, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h[0]) return fail(c, OMM_E_NONFINITE, std::string(names[i]) + " has a non-finite entry");
    if (h[1]) return fail(c, OMM_E_ASYMMETRIC, std::string(names[i]) + " is not symmetric");
  }
  return load_inputs(c, dH, dS, dT, false);
}

int omm_minimize(omm_ctx* c, const double* C0, double eta, double tau, double tol, int max_iter) {
  if (C0 && c) {
    const int64_t mn = c->M * c->N;
    for (int64_t i = 0; i < mn; ++i)
      if (!std::isfinite(C0[i])) return fail(c, OMM_E_NONFINITE, "C0 has a non-finite entry");
  }
  return minimize_impl(c, C0, false, eta, tau, tol, max_iter);
}

int omm_minimize_device(omm_ctx* c, const double* dC0, double eta, double tau, double tol,
                        int max_iter) {
  return minimize_impl(c, dC0, true, eta, tau, tol, max_iter);
}

// ---- complex Hermitian problems through the exact real embedding --------------------------
// Row form: a complex row vector c = a + i b times X = A + i B (A symmetric, B antisymmetric)
// is [a, b] [[A, B], [-B, A]] in real terms, and i c is the row [-b, a]. The embedded operators
// are real symmetric of size 2 Nc; every complex Wannier function c contributes the two rows
// [Re c, Im c] and [-Im c, Re c], so the real problem has 2 Mc rows, each complex eigenvalue
// appears twice and the real functional is twice the complex one.

int omm_create_complex(int64_t N, int64_t M, omm_ctx** out) {
  if (!out) return OMM_E_ARG;
  *out = nullptr;
  if (N <= 0 || M <= 0 || M > N || N > ((int64_t)1 << 29)) return OMM_E_ARG;
  const int r = omm_create(2 * N, 2 * M, out);
  if (r != OMM_OK) return r;
  (*out)->cplx = true;
  (*out)->Nc = N;
  (*out)->Mc = M;
  return OMM_OK;
}

int omm_set_HS_complex(omm_ctx* c, const double* H_re, const double* H_im, const double* S_re,
                       const double* S_im, const double* T_re, const double* T_im) {
  if (!c) return OMM_E_ARG;
  if (!c->cplx) return fail(c, OMM_E_STATE, "not a complex context (omm_create_complex)");
  if (!H_re || !S_re) return fail(c, OMM_E_ARG, "the real parts of H and S are required");
  if (!T_re && T_im) return fail(c, OMM_E_ARG, "T_im without T_re");
  std::vector<double> H, S, T;
  embed_operator(H_re, H_im, c->Nc, H);
  embed_operator(S_re, S_im, c->Nc, S);
  if (T_re) embed_operator(T_re, T_im, c->Nc, T);
  // the embedding is symmetric exactly when the input is Hermitian: omm_set_HS checks it
  return omm_set_HS(c, H.data(), S.data(), T_re ? T.data() : nullptr);
}

int omm_minimize_complex(omm_ctx* c, const double* C0_re, const double* C0_im, double eta,
                         double tau, double tol, int max_iter) {
  if (!c) return OMM_E_ARG;
  if (!c->cplx) return fail(c, OMM_E_STATE, "not a complex context (omm_create_complex)");
  if (!C0_re) return omm_minimize(c, nullptr, eta, tau, tol, max_iter);
  std::vector<double> C;
  embed_rows(C0_re, C0_im, c->Mc, c->Nc, C);
  return omm_minimize(c, C.data(), eta, tau, tol, max_iter);
}

int omm_density_complex(omm_ctx* c, double* rho_re, double* rho_im) {
  if (!c || !rho_re || !rho_im) return c ? fail(c, OMM_E_ARG, "null output") : OMM_E_ARG;
  if (!c->cplx) return fail(c, OMM_E_STATE, "not a complex context (omm_create_complex)");
  TRY(need_minimized(c));
  const int64_t n = c->Nc, n2 = 2 * n;
  TRY(dalloc(c, &c->nn_scratch, (size_t)n2 * n2));
  TRY(ct_x_c(c, c->SW, 2.0, true, c->nn_scratch));
  // rho = rho_hat[:n, :n] + i rho_hat[:n, n:] (the first n rows of the embedded density)
  std::vector<double> top((size_t)n * n2);
  HIPCHK(c, hipMemcpyAsync(top.data(), c->nn_scratch, top.size() * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      rho_re[i * n + j] = top[i * n2 + j];
      rho_im[i * n + j] = top[i * n2 + j + n];
    }
  return OMM_OK;
}

int omm_energy(omm_ctx* c, double* E) {
  if (!c || !E) return c ? fail(c, OMM_E_ARG, "E is null") : OMM_E_ARG;
  TRY(need_minimized(c));
  *E = c->st_host->E * (c->cplx ? 0.5 : 1.0);
  return OMM_OK;
}

int omm_density_device(omm_ctx* c, double* d_rho) {
  if (!c || !d_rho) return c ? fail(c, OMM_E_ARG, "null output") : OMM_E_ARG;
  TRY(need_minimized(c));
  TRY(ct_x_c(c, c->SW, 2.0, true, d_rho));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return OMM_OK;
}

int omm_edm_device(omm_ctx* c, double* d_edm) {
  if (!c || !d_edm) return c ? fail(c, OMM_E_ARG, "null output") : OMM_E_ARG;
  TRY(need_minimized(c));
  TRY(ct_x_c(c, c->HW, 0.0, false, d_edm));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return OMM_OK;
}

static int to_host_nn(omm_ctx* c, double* host, int (*fn)(omm_ctx*, double*)) {
  TRY(dalloc(c, &c->nn_scratch, (size_t)c->N * c->N));
  TRY(fn(c, c->nn_scratch));
  HIPCHK(c, hipMemcpy(host, c->nn_scratch, (size_t)c->N * c->N * sizeof(double),
                      hipMemcpyDeviceToHost));
  return OMM_OK;
}

int omm_density(omm_ctx* c, double* rho) {
  if (!c || !rho) return c ? fail(c, OMM_E_ARG, "null output") : OMM_E_ARG;
  return to_host_nn(c, rho, omm_density_device);
}

int omm_edm(omm_ctx* c, double* edm) {
  if (!c || !edm) return c ? fail(c, OMM_E_ARG, "null output") : OMM_E_ARG;
  return to_host_nn(c, edm, omm_edm_device);
}

int omm_backward_device(omm_ctx* c, double gE, double* d_gH, double* d_gS) {
  if (!c || !d_gH || !d_gS) return c ? fail(c, OMM_E_ARG, "null output") : OMM_E_ARG;
  if (d_gH == d_gS) return fail(c, OMM_E_ARG, "d_gH and d_gS must not alias");
  TRY(need_minimized(c));
  const int64_t nn = c->N * c->N;
  TRY(ct_x_c(c, c->SW, 2.0, true, d_gH));   // rho
  TRY(ct_x_c(c, c->HW, 0.0, false, d_gS));  // EDM
  HIPCHK(c, axpby_f64(d_gS, d_gH, d_gS, -gE, -gE * c->eta_last, nn, c->stream));
  HIPCHK(c, scale_f64(d_gH, gE, nn, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return OMM_OK;
}

int omm_get_C(omm_ctx* c, double* C) {
  if (!c || !C) return c ? fail(c, OMM_E_ARG, "null output") : OMM_E_ARG;
  const double* Cb = nullptr;
  TRY(c_original(c, &Cb));
  HIPCHK(c, hipMemcpyAsync(C, Cb, (size_t)c->M * c->N * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return OMM_OK;
}

int omm_get_subspace(omm_ctx* c, double* HW, double* SW) {
  if (!c) return OMM_E_ARG;
  TRY(need_minimized(c));
  const size_t b = (size_t)c->M * c->M * sizeof(double);
  if (HW) HIPCHK(c, hipMemcpyAsync(HW, c->HW, b, hipMemcpyDeviceToHost, c->stream));
  if (SW) HIPCHK(c, hipMemcpyAsync(SW, c->SW, b, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return OMM_OK;
}

int omm_get_preconditioner(omm_ctx* c, double* P) {
  if (!c || !P) return c ? fail(c, OMM_E_ARG, "null output") : OMM_E_ARG;
  if (c->p_kind <= 0 || !c->P) return fail(c, OMM_E_STATE, "no preconditioner has been built");
  HIPCHK(c, hipMemcpyAsync(P, c->P, (size_t)c->N * c->N * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return OMM_OK;
}

int omm_stats(omm_ctx* c, int* iters, double* last_rel) {
  if (!c) return OMM_E_ARG;
  if (iters) *iters = c->iters;
  if (last_rel) *last_rel = c->last_rel;
  return OMM_OK;
}

int omm_phase_stats(omm_ctx* c, int* mixed_iters, int* fp64_iters) {
  if (!c) return OMM_E_ARG;
  const int last = c->iters - c->iters_before;  // line searches of the active phase
  if (mixed_iters) *mixed_iters = c->phase_prec != OMM_FP64 ? last : c->iters_before;
  if (fp64_iters) *fp64_iters = c->phase_prec == OMM_FP64 ? last : 0;
  return OMM_OK;
}

int omm_energy_trace(omm_ctx* c, double* buf, int cap, int* n) {
  if (!c || (!buf && cap > 0)) return c ? fail(c, OMM_E_ARG, "null buffer") : OMM_E_ARG;
  const int k = (int)c->trace_host.size() < cap ? (int)c->trace_host.size() : cap;
  for (int i = 0; i < k; ++i) buf[i] = c->trace_host[i] * (c->cplx ? 0.5 : 1.0);
  if (n) *n = (int)c->trace_host.size();
  return OMM_OK;
}

int omm_iterate(omm_ctx* c, int count, double tol) {
  if (!c) return OMM_E_ARG;
  if (count < 0 || !(tol >= 0.0)) return fail(c, OMM_E_ARG, "need count >= 0 and tol >= 0");
  if (!c->phase_active) return fail(c, OMM_E_STATE, "no active minimization to continue");
  int done = 0;
  if (c->phase_mixed64) {
    TRY(mixed64_iterate(c, tol, count, false, &done));
    c->c_prec = OMM_FP64;
  } else if (c->phase_prec == OMM_FP64) {
    TRY(phase_iterate<double>(c, c->w64, CF64, c->Hs, c->S, c->p_kind > 0 ? c->P : nullptr, tol,
                              count, &done));
    c->c_prec = OMM_FP64;
  } else {
    TRY(phase_iterate<float>(c, c->w32, compute_of(c->phase_prec), c->Hs32, c->S32,
                             c->p_kind > 0 ? c->P32 : nullptr, tol, count, &done));
    c->c_prec = c->phase_prec;
  }
  c->iters = c->iters_before + c->st_host->iter;
  c->trace_n = c->trace_off + c->st_host->iter + 1;
  c->last_rel = c->st_host->rel_change;
  c->trace_host.assign((size_t)c->trace_n, 0.0);
  HIPCHK(c, hipMemcpyAsync(c->trace_host.data(), c->trace, c->trace_n * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return status_of_done(c, done);
}

int omm_set_profiling(omm_ctx* c, int on) {
  if (!c) return OMM_E_ARG;
  TRY(prof_collect(c));
  drop_graph(c);
  c->prof = on != 0;
  c->ev_used = 0;
  for (int i = 0; i < NSTAGE; ++i) c->stage_ms[i] = 0.0;
  c->prof_iters = 0;
  return OMM_OK;
}

int omm_stage_times(omm_ctx* c, double* ms, int cap, int* iters) {
  if (!c || (!ms && cap > 0)) return c ? fail(c, OMM_E_ARG, "null buffer") : OMM_E_ARG;
  TRY(prof_collect(c));
  for (int i = 0; i < cap && i < NSTAGE; ++i) ms[i] = c->stage_ms[i];
  if (iters) *iters = c->prof_iters;
  return NSTAGE;
}

const char* omm_last_error(const omm_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

}  // extern "C"

// ---- the backward pass without allocation ------------------------------------------------------
// omm_backward_device_noalloc computes what omm_backward_device does through a fixed scratch
// array instead of the context's buffers or any allocation: rho = 2 C^T (2I - SW) C and
// EDM = 2 C^T HW C are accumulated over chunks of R rows of C,
//   Z = 2 C[r0:r1] - SW[r0:r1] C  then  d_gH += 2 gE C[r0:r1]^T Z,
//   Z = HW[r0:r1] C               then  d_gS -= 2 gE C[r0:r1]^T Z,
// with Z (R x N) in `scratch`, and finally d_gS -= eta d_gH. R = min(M, capacity / N) must be at
// least NOALLOC_MIN_ROWS (or M), which bounds N. Every call on a device shares that device's
// copy of the array: calls that overlap on one GPU race.
namespace {
constexpr int64_t NOALLOC_SCRATCH_DOUBLES = (int64_t)1 << 21;  // 16 MiB per device
constexpr int64_t NOALLOC_MIN_ROWS = 64;
__device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];
constexpr int NOALLOC_MAX_DEVICES = 64;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
std::mutex g_scratch_mu;

// The device address of this device's copy of `scratch` (looked up once per device).
int scratch_address(omm_ctx* c, double** out) {
  int dev = 0;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(c, OMM_E_HIP, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, OMM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return OMM_OK;
}
}  // namespace

extern "C" int omm_backward_device_noalloc(omm_ctx* c, double gE, double* d_gH, double* d_gS) {
  if (!c || !d_gH || !d_gS) return c ? fail(c, OMM_E_ARG, "null output") : OMM_E_ARG;
  if (d_gH == d_gS) return fail(c, OMM_E_ARG, "d_gH and d_gS must not alias");
  const int64_t M = c->M, N = c->N;
  const int64_t R = std::min<int64_t>(M, NOALLOC_SCRATCH_DOUBLES / N);
  if (R < std::min<int64_t>(M, NOALLOC_MIN_ROWS))
    return fail(c, OMM_E_ARG, "omm_backward_device_noalloc: N = " + std::to_string(N) +
                                  " exceeds its scratch (N <= " +
                                  std::to_string(NOALLOC_SCRATCH_DOUBLES / NOALLOC_MIN_ROWS) +
                                  "); use omm_backward_device");
  TRY(need_minimized(c));
  if (c->c_flavour == OMM_FLAVOUR_CHOLESKY)
    return fail(c, OMM_E_STATE, "omm_backward_device_noalloc: the Cholesky flavour needs C~ L^-1 "
                                "in an allocated buffer; use omm_backward_device");
  TRY(c64(c));  // converts into the context's own FP64 C (no allocation)
  double* Z = nullptr;
  TRY(scratch_address(c, &Z));
  const double* C = c->w64.C;
  // FP64 tile 0 (128 x 128), no split-K: no workspace
  const GemmDesc dz{CF64, T_F64, T_F64, T_F64, T_F64, KC, RC, 0, 1};   // Z = X[r0:r1] C
  const GemmDesc dc{CF64, T_F64, T_F64, T_F64, T_F64, RC, RC, 0, 1};   // out += C[r0:r1]^T Z
  for (int64_t r0 = 0; r0 < M; r0 += R) {
    const int rows = (int)std::min<int64_t>(R, M - r0);
    for (int which = 0; which < 2; ++which) {
      const double* X = which == 0 ? c->SW : c->HW;
      double* out = which == 0 ? d_gH : d_gS;
      // which 0: Z = 2 C[r0:r1] - SW[r0:r1] C;  which 1: Z = HW[r0:r1] C
      GemmOp oz = make_op(rows, (int)N, (int)M, X + r0 * M, M, C, N, Z, N,
                          which == 0 ? -1.0 : 1.0, which == 0 ? C + r0 * N : nullptr, N,
                          which == 0 ? 2.0 : 0.0);
      HIPCHK(c, gemm_launch(dz, &oz, 1, nullptr, nullptr, 0, c->stream));
      // out (+)= (+-2 gE) C[r0:r1]^T Z: A(m, k) = C[r0 + k][m], B(k, n) = Z[k][n]
      const double sc = which == 0 ? 2.0 * gE : -2.0 * gE;
      GemmOp oc = make_op((int)N, (int)N, rows, C + r0 * N, N, Z, N, out, N, sc,
                          r0 > 0 ? out : nullptr, N, r0 > 0 ? 1.0 : 0.0);
      HIPCHK(c, gemm_launch(dc, &oc, 1, nullptr, nullptr, 0, c->stream));
    }
  }
  // dE/dS = -EDM - eta rho: d_gS = gE (-EDM) - eta (gE rho)
  HIPCHK(c, axpby_f64(d_gS, d_gH, d_gS, 1.0, -c->eta_last, N * N, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return OMM_OK;
}
