// Batched entry points: many independent (H, S) systems of uneven size.
//
// Each system gets its own context on a shared stream; systems are minimized one after
// another with the FP32 MFMA plan. This is the correctness baseline of the batched interface.
#include <string>
#include <vector>

#include "../../include/omm.h"

struct omm_batch {
  std::vector<omm_ctx*> sys;
  std::vector<int> iters;
  std::vector<double> E;
  std::string err;
};

namespace {
int bfail(omm_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  return code;
}
}  // namespace

extern "C" {

int omm_batch_create(int nsys, const int64_t* N, const int64_t* M, omm_batch** out) {
  if (!out) return OMM_E_ARG;
  *out = nullptr;
  if (nsys <= 0 || !N || !M) return OMM_E_ARG;
  omm_batch* b = new omm_batch();
  for (int i = 0; i < nsys; ++i) {
    omm_ctx* c = nullptr;
    int r = omm_create(N[i], M[i], &c);
    if (r != OMM_OK) {
      for (omm_ctx* x : b->sys) omm_destroy(x);
      delete b;
      return r;
    }
    omm_set_precision(c, OMM_FP32, 0);
    b->sys.push_back(c);
  }
  b->iters.assign(nsys, 0);
  b->E.assign(nsys, 0.0);
  *out = b;
  return OMM_OK;
}

int omm_batch_destroy(omm_batch* b) {
  if (!b) return OMM_E_ARG;
  for (omm_ctx* c : b->sys) omm_destroy(c);
  delete b;
  return OMM_OK;
}

int omm_batch_set_HS(omm_batch* b, int i, const double* H, const double* S, const double* T) {
  if (!b) return OMM_E_ARG;
  if (i < 0 || i >= (int)b->sys.size()) return bfail(b, OMM_E_ARG, "system index out of range");
  int r = omm_set_HS(b->sys[i], H, S, T);
  if (r != OMM_OK) return bfail(b, r, omm_last_error(b->sys[i]));
  return OMM_OK;
}

int omm_batch_minimize(omm_batch* b, const double* const* C0, const double* eta, const double* tau,
                       double tol, int max_iter) {
  if (!b || !eta || !tau) return b ? bfail(b, OMM_E_ARG, "eta and tau are required") : OMM_E_ARG;
  int worst = OMM_OK;
  for (size_t i = 0; i < b->sys.size(); ++i) {
    int r = omm_minimize(b->sys[i], C0 ? C0[i] : nullptr, eta[i], tau[i], tol, max_iter);
    if (r < 0) return bfail(b, r, "system " + std::to_string(i) + ": " + omm_last_error(b->sys[i]));
    if (r > 0) worst = r;
    omm_stats(b->sys[i], &b->iters[i], nullptr);
    omm_energy(b->sys[i], &b->E[i]);
  }
  return worst;
}

int omm_batch_energy(omm_batch* b, double* E) {
  if (!b || !E) return OMM_E_ARG;
  for (size_t i = 0; i < b->E.size(); ++i) E[i] = b->E[i];
  return OMM_OK;
}

int omm_batch_iterations(omm_batch* b, int* iters) {
  if (!b || !iters) return OMM_E_ARG;
  for (size_t i = 0; i < b->iters.size(); ++i) iters[i] = b->iters[i];
  return OMM_OK;
}

int omm_batch_get_C(omm_batch* b, int i, double* C) {
  if (!b || !C) return OMM_E_ARG;
  if (i < 0 || i >= (int)b->sys.size()) return bfail(b, OMM_E_ARG, "system index out of range");
  return omm_get_C(b->sys[i], C);
}

const char* omm_batch_last_error(const omm_batch* b) {
  if (!b) return "null batch";
  return b->err.c_str();
}

}  // extern "C"
