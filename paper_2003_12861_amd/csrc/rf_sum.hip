// rf_sum.hip -- combined likelihoods: independent terms that share
// parameters, times Gaussian constraint factors (Section 3: combined
// measurements of parameters such as a signal strength).
//
//   NLL(theta) = sum_t NLL_t(theta[map_t]) + sum_c (theta[k_c] - m_c)^2 / (2 w_c^2)
//
// An evaluation enqueues every term's own NLL+gradient kernel on the stream
// (each writes its result block in device memory), then one workgroup of up
// to four wavefronts adds them.  Lane k reads global parameter k's gradient
// entries through an inverse map (the addresses of the entries inside the
// terms' result blocks, terms in order and each term's parameters in order,
// built on the host and uploaded when the sum or a result block changes)
// and loads them sixteen at a time; lane 0 adds the NLLs and the bad-event
// counts in term order; the constraints come last.  The order is fixed, so
// results repeat bit for bit.  The result goes to device memory and, word
// by word with system-scope stores, to mapped host memory, which the
// synchronous call polls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device/rf_dev.h"
#include "rf_internal.h"

#define RF_SUM_MAXTERMS 16
#define RF_SUM_MAXP 256  // global parameters at most (one lane each in the combining kernel)

namespace {

struct SumArgs {
  const double* res[RF_SUM_MAXTERMS];  // each term's device result block [nll, grad[P_t], ...]
  int32_t nbad[RF_SUM_MAXTERMS];       // index of its bad-event count in the block (-1: none)
  const double* const* inv;            // parameter k's gradient entries are inv[inv_off[k] ..
                                       //   inv_off[k + 1]), the addresses of the terms' gradient
                                       //   entries mapped to k, terms in order, parameters in order
  int32_t nterms, P, nc, pad_;
  int32_t inv_off[RF_SUM_MAXP + 2];    // [P + 1] used (carried here: one memory round trip less)
  int32_t ck[RF_MAX_PARAMS];           // constraint c: parameter index,
  double cval[RF_MAX_PARAMS];          //   the parameter's value at this point,
  double cmean[RF_MAX_PARAMS];         //   mean,
  double cinv2[RF_MAX_PARAMS];         //   1 / width^2
  double* out;                         // [nll, grad[P], n_bad]
  double* hout;                        // mapped host copy of out
};

static_assert(sizeof(SumArgs) <= 4096, "the combining kernel's arguments stay within 4 KiB");

// Every load of a lane is independent of the others (addresses from the
// inverse map, 16 at a time), so a lane waits for about two memory round
// trips (the entry addresses, then the entries), not one per map entry.
__global__ __launch_bounds__(RF_SUM_MAXP) void rf_k_sum(const SumArgs a) {
  const int k = threadIdx.x;  // one global parameter per lane
  if (k < a.P) {
    const int beg = a.inv_off[k], end = a.inv_off[k + 1];
    double g = 0.0;
    for (int b0 = beg; b0 < end; b0 += 16) {
      double v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = b0 + i < end ? *a.inv[b0 + i] : 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) g += v[i];
    }
    for (int c = 0; c < a.nc; ++c)
      if (a.ck[c] == k) g += (a.cval[c] - a.cmean[c]) * a.cinv2[c];
    a.out[1 + k] = g;
    rf_store_host(a.hout + 1 + k, g);
  }
  if (k == 0) {
    double tn[RF_SUM_MAXTERMS], tb[RF_SUM_MAXTERMS];
#pragma unroll
    for (int t = 0; t < RF_SUM_MAXTERMS; ++t) {
      tn[t] = t < a.nterms ? a.res[t][0] : 0.0;
      tb[t] = t < a.nterms && a.nbad[t] >= 0 ? a.res[t][a.nbad[t]] : 0.0;
    }
    double nll = 0.0, bad = 0.0;
#pragma unroll
    for (int t = 0; t < RF_SUM_MAXTERMS; ++t) {
      nll += tn[t];
      bad += tb[t];
    }
    for (int c = 0; c < a.nc; ++c) {
      const double d = a.cval[c] - a.cmean[c];
      nll += 0.5 * d * d * a.cinv2[c];
    }
    a.out[0] = nll;
    a.out[1 + a.P] = bad;
    rf_store_host(a.hout, nll);
    rf_store_host(a.hout + 1 + a.P, bad);
  }
}

}  // namespace

struct rf_sum {
  int P = 0;
  std::vector<double> lo, hi;  // bounds, narrowed by the terms'
  struct Term {
    rf_program* p = nullptr;
    rf_binned* b = nullptr;
    std::vector<int32_t> map;
    const double* res = nullptr;  // its result block when the inverse map was built
  };
  std::vector<Term> terms;
  std::vector<int32_t> ck;
  std::vector<double> cmean, cwidth;
  // device state, taken at the first evaluation
  int device = -1;
  std::vector<int32_t> inv_off;       // inverse map (see SumArgs): the offsets, passed with
                                      // each launch, and the entry addresses, uploaded after a change
  const double** d_inv = nullptr;
  size_t inv_cap = 0;
  bool dirty = true;  // the maps changed since they were uploaded
  double* d_out = nullptr;
  double* h_out = nullptr;
  double* d_hout = nullptr;
  void* last_stream = nullptr;  // stream of the previous combining kernel (see order_launch)
  bool launched = false;
};

using namespace rf;

namespace {

int add_term(rf_sum* s, rf_program* p, rf_binned* b, const int32_t* map, int np,
             const std::vector<double>& tlo, const std::vector<double>& thi) {
  if (!map) return fail(RF_E_INVALID, "NULL argument");
  if ((int)s->terms.size() >= RF_SUM_MAXTERMS) return fail(RF_E_INVALID, "at most 16 terms in a sum");
  for (const auto& t : s->terms)
    if ((p && t.p == p) || (b && t.b == b)) return fail(RF_E_INVALID, "the term is already in this sum");
  if (np < 1 || np > RF_MAX_PARAMS) return fail(RF_E_INVALID, "the term has no parameters");
  std::vector<double> lo = s->lo, hi = s->hi;
  for (int j = 0; j < np; ++j) {
    const int k = map[j];
    if (k < 0 || k >= s->P) return fail(RF_E_INVALID, "map index outside [0, n_params)");
    lo[k] = std::max(lo[k], tlo[j]);
    hi[k] = std::min(hi[k], thi[j]);
    if (!(lo[k] <= hi[k])) return fail(RF_E_INVALID, "the bounds of a shared parameter do not overlap");
  }
  rf_sum::Term t;
  t.p = p;
  t.b = b;
  t.map.assign(map, map + np);
  s->terms.push_back(t);
  s->lo = lo;
  s->hi = hi;
  s->dirty = true;
  return RF_OK;
}

// device buffers at the first evaluation; the maps again after a change
int prepare(rf_sum* s) {
  hipError_t e;
  if (!s->d_out) {
    if ((e = hipGetDevice(&s->device)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    if ((e = hipMalloc(&s->d_out, sizeof(double) * (RF_SUM_MAXP + 2))) != hipSuccess) return hip_fail(e, "hipMalloc");
    if ((e = hipHostMalloc(&s->h_out, sizeof(double) * (RF_SUM_MAXP + 2), hipHostMallocMapped | hipHostMallocCoherent)) !=
            hipSuccess ||
        (e = hipHostGetDevicePointer((void**)&s->d_hout, s->h_out, 0)) != hipSuccess)
      return hip_fail(e, "mapped result buffer");
  }
  if (!s->dirty) return RF_OK;
  // the inverse map: for each global parameter, the device addresses of the
  // terms' gradient entries mapped to it, terms in order, parameters in order
  std::vector<int32_t> off(s->P + 1, 0);
  for (const auto& t : s->terms)
    for (int32_t k : t.map) ++off[k + 1];
  for (int k = 0; k < s->P; ++k) off[k + 1] += off[k];
  std::vector<const double*> inv(off[s->P] > 0 ? off[s->P] : 1);
  {
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (const auto& t : s->terms) {
      if (!t.res) return fail(RF_E_STATE, "a term has no result block (program not bound or not loaded)");
      for (size_t j = 0; j < t.map.size(); ++j) inv[fill[t.map[j]]++] = t.res + 1 + j;
    }
  }
  // a combining kernel still in flight reads the old map
  if (s->launched && (e = hipStreamSynchronize((hipStream_t)s->last_stream)) != hipSuccess)
    return hip_fail(e, "hipStreamSynchronize (previous stream)");
  if (inv.size() > s->inv_cap) {
    if (s->d_inv) (void)hipFree(s->d_inv);
    s->d_inv = nullptr;
    s->inv_cap = 0;
    if ((e = hipMalloc(&s->d_inv, sizeof(const double*) * inv.size())) != hipSuccess) return hip_fail(e, "hipMalloc");
    s->inv_cap = inv.size();
  }
  if ((e = hipMemcpy(s->d_inv, inv.data(), sizeof(const double*) * inv.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy");
  s->inv_off = off;
  s->dirty = false;
  return RF_OK;
}

}  // namespace

extern "C" {

int rf_sum_new(int32_t n_params, const double* lo, const double* hi, rf_sum** out) {
  if (!out) return fail(RF_E_INVALID, "NULL argument");
  *out = nullptr;
  if (n_params < 1 || n_params > RF_SUM_MAXP) return fail(RF_E_INVALID, "n_params must be in 1..256");
  rf_sum* s = new rf_sum();
  s->P = n_params;
  s->lo.assign(n_params, -INFINITY);
  s->hi.assign(n_params, INFINITY);
  for (int k = 0; k < n_params; ++k) {
    if (lo) s->lo[k] = lo[k];
    if (hi) s->hi[k] = hi[k];
    if (std::isnan(s->lo[k]) || std::isnan(s->hi[k]) || !(s->lo[k] <= s->hi[k])) {
      delete s;
      return fail(RF_E_INVALID, "bounds must satisfy lo <= hi");
    }
  }
  *out = s;
  return RF_OK;
}

void rf_sum_free(rf_sum* s) {
  if (!s) return;
  if (s->d_inv) (void)hipFree(s->d_inv);
  if (s->d_out) (void)hipFree(s->d_out);
  if (s->h_out) (void)hipHostFree(s->h_out);
  delete s;
}

int rf_sum_add_program(rf_sum* s, rf_program* p, const int32_t* map) {
  if (!s || !p) return fail(RF_E_INVALID, "NULL argument");
  return add_term(s, p, nullptr, map, p->L.n_params, p->L.plo, p->L.phi);
}

int rf_sum_add_binned(rf_sum* s, rf_binned* b, const int32_t* map) {
  if (!s || !b) return fail(RF_E_INVALID, "NULL argument");
  const int np = binned_n_params(b);
  std::vector<double> lo(np, -INFINITY), hi(np, INFINITY);
  lo[0] = 0.0;  // the signal strength
  return add_term(s, nullptr, b, map, np, lo, hi);
}

int rf_sum_add_constraint(rf_sum* s, int32_t k, double mean, double width) {
  if (!s) return fail(RF_E_INVALID, "NULL argument");
  if (k < 0 || k >= s->P) return fail(RF_E_INVALID, "parameter index outside [0, n_params)");
  if (!std::isfinite(mean) || !(width > 0) || !std::isfinite(width))
    return fail(RF_E_INVALID, "a constraint needs a finite mean and a finite width > 0");
  if ((int)s->ck.size() >= RF_MAX_PARAMS) return fail(RF_E_INVALID, "at most 64 constraints");
  s->ck.push_back(k);
  s->cmean.push_back(mean);
  s->cwidth.push_back(width);
  return RF_OK;
}

int rf_sum_nll_grad(rf_sum* s, const double* theta, double* nll, double* grad, int64_t* n_bad, void* stream) {
  if (!s || !theta || !nll || !grad) return fail(RF_E_INVALID, "NULL argument");
  const int P = s->P;
  for (int k = 0; k < P; ++k) {
    if (!std::isfinite(theta[k])) return fail(RF_E_DOMAIN, "theta must be finite");
    if (theta[k] < s->lo[k] || theta[k] > s->hi[k]) return fail(RF_E_DOMAIN, "theta outside its bounds");
  }
  // a term's result block moves when its program is bound to more events:
  // rebuild the inverse map then
  for (auto& t : s->terms) {
    const double* r = t.p ? rf_program_result(t.p) : rf_binned_result(t.b);
    if (r != t.res) {
      t.res = r;
      s->dirty = true;
    }
  }
  int rc = prepare(s);
  if (rc) return rc;
  SumArgs a;
  memset(&a, 0, sizeof a);
  double th[RF_MAX_PARAMS];
  for (size_t t = 0; t < s->terms.size(); ++t) {
    const rf_sum::Term& term = s->terms[t];
    const int np = (int)term.map.size();
    for (int j = 0; j < np; ++j) th[j] = theta[term.map[j]];
    if (term.p) {
      if (term.p->loaded && term.p->device != s->device) return fail(RF_E_INVALID, "a term lives on another device");
      rc = rf_nll_grad_async(term.p, th, stream);
      a.res[t] = rf_program_result(term.p);
      a.nbad[t] = 1 + np;
    } else {
      rc = rf_binned_nll_grad_async(term.b, th, stream);
      a.res[t] = rf_binned_result(term.b);
      a.nbad[t] = -1;
    }
    if (rc) return rc;
  }
  memcpy(a.inv_off, s->inv_off.data(), sizeof(int32_t) * (P + 1));
  a.inv = s->d_inv;
  a.nterms = (int32_t)s->terms.size();
  a.P = P;
  a.nc = (int32_t)s->ck.size();
  for (int c = 0; c < a.nc; ++c) {
    a.ck[c] = s->ck[c];
    a.cval[c] = theta[s->ck[c]];
    a.cmean[c] = s->cmean[c];
    a.cinv2[c] = 1.0 / (s->cwidth[c] * s->cwidth[c]);
  }
  a.out = s->d_out;
  a.hout = s->d_hout;
  if ((rc = order_launch(s->last_stream, s->launched, stream))) return rc;
  arm_result(s->h_out, P + 2);
  hipLaunchKernelGGL(rf_k_sum, dim3(1), dim3((P + 63) / 64 * 64), 0, (hipStream_t)stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "combining kernel launch");
  if ((rc = wait_result(s->h_out, P + 2, stream, nullptr))) return rc;
  const int64_t bad = (int64_t)s->h_out[1 + P];
  if (n_bad) *n_bad = bad;
  const bool finite = std::isfinite(s->h_out[0]);
  *nll = (bad || !finite) ? INFINITY : s->h_out[0];
  for (int k = 0; k < P; ++k) grad[k] = (bad || !finite) ? NAN : s->h_out[1 + k];
  if (bad) return fail(RF_E_NONFINITE, std::to_string(bad) + " events with p <= 0 or non-finite p");
  if (!finite) return fail(RF_E_NONFINITE, "non-finite NLL (a term's NLL is not finite)");
  return RF_OK;
}

int rf_sum_fit_bfgs(rf_sum* s, const double* theta0, double edm_tol, int32_t max_iter, double* theta_out,
                    double* sigma_out, double* cov_out, double* info_out, void* stream) {
  if (!s) return fail(RF_E_INVALID, "NULL argument");
  Objective obj;
  obj.P = s->P;
  obj.lo = s->lo;
  obj.hi = s->hi;
  obj.eval = [s, stream](const double* x, double* f, double* g) {
    return rf_sum_nll_grad(s, x, f, g, nullptr, stream);
  };
  return bfgs_fit(obj, theta0, nullptr, edm_tol, max_iter, theta_out, sigma_out, cov_out, info_out);
}

}  // extern "C"
